"""Batched solve (fj_solve_batched) against the FP64 oracle, and its recorded
hipGraph against eager enqueueing.

The batch mixes directed/weighted and undirected single-vector graphs with a
multi-vector item; every vector must meet the same certificate as fj_solve
(Lemma 7 with Alg. 2's shift), and the measures must match the oracle's on
the exact solution.
"""
import numpy as np
import pytest

import oracle
import synth
from tests import graphs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"
EPS = 1e-6


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _dev(g):
    rp = torch.from_numpy(g.row_ptr).to(DEV)
    col = torch.from_numpy(g.col).to(DEV)
    w = None if g.w is None else torch.from_numpy(g.w).to(DEV)
    return (rp, col, w, g.directed)


def _items():
    single = [
        synth.chung_lu(3000, 12000, 2.3, 501),
        synth.chung_lu(5000, 40000, 2.1, 502, directed=True, weighted=True),
        synth.barabasi_albert(1500, 4, 503),
        graphs.random_graph(65, 0.1, 504),
        synth.chung_lu(4000, 20000, 2.2, 505, weighted=True),
    ]
    multi = synth.chung_lu(20000, 100000, 2.3, 510)
    return single, multi


def _fill(B, single, multi, k):
    ss = []
    for i, g in enumerate(single):
        s = synth.opinions(g.n, ["uniform", "bimodal", "beta", "exp", "pareto"][i], 600 + i)
        B.input(i).copy_(torch.from_numpy(s))
        ss.append(s)
    sm = np.stack([synth.opinions(multi.n, "beta", 700 + q, a=2, b=2) for q in range(k)], axis=1)
    B.input(len(single)).copy_(torch.from_numpy(np.ascontiguousarray(sm)))
    return ss, sm


def _check(g, s, z, zt):
    epsp = 0.5 * EPS
    assert np.all(np.abs(z - zt) <= epsp * (zt + 1e-5) * (1 + 1e-9) + 1e-15)
    assert oracle.certificate(g, s, z, EPS) <= 1.0 + 1e-9


def test_batched_matches_oracle():
    import paper_2507_14864_amd as fj
    single, multi = _items()
    k = 5
    B = fj.Batch([_dev(g) for g in single] + [_dev(multi)], [1] * len(single) + [k], eps=EPS, omega=1.4)
    ss, sm = _fill(B, single, multi, k)
    stats, mets = B.solve()
    for i, g in enumerate(single):
        zt = oracle.exact(g, ss[i])
        z = B.output(i).cpu().numpy()
        _check(g, ss[i], z, zt)
        assert stats[i]["certified"] == 1 and stats[i]["max_ratio"] <= 1.0
        mo = oracle.metrics(g, ss[i], zt)
        for key in "PDIC":
            assert abs(mets[i][0][key] - mo[key]) <= 1e-5 * abs(mo[key]), (i, key)
    zm = B.output(len(single)).cpu().numpy()
    assert stats[-1]["certified"] == 1
    for q in range(k):
        zt = oracle.exact(multi, sm[:, q])
        _check(multi, sm[:, q], zm[:, q], zt)
        mo = oracle.metrics(multi, sm[:, q], zt)
        for key in "PDIC":
            assert abs(mets[-1][q][key] - mo[key]) <= 1e-5 * abs(mo[key]), (q, key)
        # the measures reported for the returned z are those of z itself
        mz = oracle.metrics(multi, sm[:, q], zm[:, q])
        for key in "PDIC":
            assert abs(mets[-1][q][key] - mz[key]) <= 1e-10 * abs(mz[key]), (q, key)


def test_multi_vector_item_agrees_with_single_solves():
    import paper_2507_14864_amd as fj
    g = synth.chung_lu(15000, 80000, 2.3, 520, directed=True, weighted=True)
    k = 64
    S = np.stack([synth.opinions(g.n, "uniform", 800 + q) for q in range(k)], axis=1)
    B = fj.Batch([_dev(g)], [k], eps=EPS, omega=1.1)
    B.input(0).copy_(torch.from_numpy(np.ascontiguousarray(S)))
    stats, _ = B.solve()
    assert stats[0]["certified"] == 1
    Z = B.output(0).cpu().numpy()
    G = fj.Graph.from_host(g, DEV, colour=True)
    for q in (0, 17, 63):
        z1, _ = fj.solve(G, torch.from_numpy(S[:, q].copy()).to(DEV), eps=EPS, omega=1.1, schedule="sor",
                         precision="fp64")
        assert np.max(np.abs(Z[:, q] - z1.cpu().numpy()) / (np.abs(z1.cpu().numpy()) + 1e-5)) <= 2 * EPS


def test_recorded_graph_replays_match_eager():
    import paper_2507_14864_amd as fj
    single, multi = _items()
    k = 3
    B = fj.Batch([_dev(g) for g in single] + [_dev(multi)], [1] * len(single) + [k], eps=EPS, omega=1.4)
    _fill(B, single, multi, k)
    info = B.tune([1.2, 1.5])
    assert info["graph_nodes"] > 0
    for key in ("omega_undirected", "omega_directed", "omega_multi"):
        assert info[key] in (1.2, 1.5)
    # eager reference: a second batch with the tuned omegas set by hand and no
    # recorded graph (kernels enqueued directly)
    E = fj.Batch([_dev(g) for g in single] + [_dev(multi)], [1] * len(single) + [k], eps=EPS, omega=1.4)
    _fill(E, single, multi, k)
    E.set_omegas(info["omega_undirected"], info["omega_directed"], info["omega_multi"])
    stats_e, mets_e = E.solve()
    z_e = [E.output(i).cpu().numpy().copy() for i in range(len(single) + 1)]
    for rep in range(3):
        junk = torch.randn(1 << 20, device=DEV)  # eager work between replays
        junk.mul_(2.0).sum().item()
        stats_g, mets_g = B.solve()
        for i in range(len(single) + 1):
            assert np.array_equal(B.output(i).cpu().numpy(), z_e[i]), (rep, i)
        for i in range(len(single) + 1):
            assert stats_g[i]["certified"] == 1
            assert stats_g[i]["rounds"] == stats_e[i]["rounds"]
            for q in range(len(mets_g[i])):
                assert mets_g[i][q] == mets_e[i][q]


def test_two_multi_vector_items_in_the_concurrent_graph():
    """Two multi-vector items (one undirected, one directed and weighted)
    beside the single-vector union: the recorded graph runs the union and the
    multi-vector items as two concurrent branches, each with its own sweep
    bookkeeping over its slots.  Its replays equal an eager batch (one chain
    on one stream) bit for bit, and sampled vectors of both items meet
    Lemma 7's bound against the oracle's exact solution."""
    import paper_2507_14864_amd as fj
    single, _ = _items()
    ma = synth.chung_lu(12000, 60000, 2.3, 530)
    mb = synth.chung_lu(9000, 50000, 2.1, 531, directed=True, weighted=True)
    ka, kb = 3, 7
    multi_items = [(ma, ka, "beta"), (mb, kb, "uniform")]

    def make():
        B = fj.Batch([_dev(g) for g in single] + [_dev(ma), _dev(mb)], [1] * len(single) + [ka, kb], eps=EPS,
                     omega=1.2)
        ss = []
        for i, g in enumerate(single):
            s = synth.opinions(g.n, "uniform", 900 + i)
            B.input(i).copy_(torch.from_numpy(s))
            ss.append(s)
        sm = []
        for j, (g, k, kind) in enumerate(multi_items):
            S = np.stack([synth.opinions(g.n, kind, 950 + 10 * j + q, a=2, b=2) if kind == "beta"
                          else synth.opinions(g.n, kind, 950 + 10 * j + q) for q in range(k)], axis=1)
            B.input(len(single) + j).copy_(torch.from_numpy(np.ascontiguousarray(S)))
            sm.append(S)
        return B, ss, sm

    B, ss, sm = make()
    info = B.tune([1.2])  # one candidate: every group at 1.2, then the graph is recorded
    assert info["graph_nodes"] > 0
    E, _, _ = make()
    E.set_omegas(1.2, 1.2, 1.2)  # no recorded graph: the eager sequence
    stats_e, mets_e = E.solve()
    nitems = len(single) + 2
    z_e = [E.output(i).cpu().numpy().copy() for i in range(nitems)]
    for rep in range(2):
        stats_g, mets_g = B.solve()
        for i in range(nitems):
            assert np.array_equal(B.output(i).cpu().numpy(), z_e[i]), (rep, i)
            assert stats_g[i]["certified"] == 1 and stats_g[i]["rounds"] == stats_e[i]["rounds"]
            assert stats_g[i]["edge_visits"] == stats_e[i]["edge_visits"]
            for q in range(len(mets_g[i])):
                assert mets_g[i][q] == mets_e[i][q]
    for j, (g, k, _) in enumerate(multi_items):
        z = B.output(len(single) + j).cpu().numpy()
        for q in (0, k - 1):
            zt = oracle.exact(g, sm[j][:, q])
            _check(g, sm[j][:, q], z[:, q], zt)
    zt = oracle.exact(single[1], ss[1])
    _check(single[1], ss[1], B.output(1).cpu().numpy(), zt)
    B.close()
    E.close()


def test_batch_rejects_bad_items():
    import paper_2507_14864_amd as fj
    g = synth.chung_lu(1000, 4000, 2.3, 530)
    bad = synth.CSRGraph(3, np.array([0, 1, 1, 1], np.int32), np.array([1], np.int32), None, False)  # asymmetric
    with pytest.raises(fj.FJError):
        fj.Batch([_dev(g), _dev(bad)], [1, 1])
    with pytest.raises((fj.FJError, ValueError)):
        fj.Batch([_dev(g)], [65])


def _all_certified_against_oracle(B, single, multi, ss, sm, k):
    stats, mets = B.results()
    for i, g in enumerate(single):
        assert stats[i]["certified"] == 1, (i, stats[i])
        _check(g, ss[i], B.output(i).cpu().numpy(), oracle.exact(g, ss[i]))
    assert stats[-1]["certified"] == 1, stats[-1]
    zm = B.output(len(single)).cpu().numpy()
    for q in range(k):
        _check(multi, sm[:, q], zm[:, q], oracle.exact(multi, sm[:, q]))
    return stats


def test_check_continues_items_beyond_the_recorded_budget():
    """After tuning, a slower relaxation factor leaves every item short of its
    certificate within the recorded budget; fj_batch_check sweeps them on from
    their estimates (Lemma 4) to the certificate."""
    import paper_2507_14864_amd as fj
    single, multi = _items()
    k = 3
    B = fj.Batch([_dev(g) for g in single] + [_dev(multi)], [1] * len(single) + [k], eps=EPS, omega=1.4)
    ss, sm = _fill(B, single, multi, k)
    info = B.tune([1.2, 1.5])
    B.set_omegas(0.4, 0.4, 0.4)  # keeps the tuned budget, drops the recording
    stats, _ = B.solve()
    short = sum(1 for st in stats if not st["certified"])
    print(f"budget {info['sweep_budget']}: {short} of {len(stats)} items short of the certificate", flush=True)
    assert short > 0
    assert B.check(extra_sweeps=4000) == 0
    stats = _all_certified_against_oracle(B, single, multi, ss, sm, k)
    assert max(st["rounds"] for st in stats) > info["sweep_budget"]


def test_opinions_swapped_after_tuning_are_certified():
    """Tuned on one set of opinions, solved on the paper's Pareto law (Sec. 6):
    every item ends certified, with fj_batch_check finishing any item the
    recorded budget did not."""
    import paper_2507_14864_amd as fj
    single, multi = _items()
    k = 3
    B = fj.Batch([_dev(g) for g in single] + [_dev(multi)], [1] * len(single) + [k], eps=EPS, omega=1.4)
    _fill(B, single, multi, k)
    B.tune([1.2, 1.5])
    ss = []
    for i, g in enumerate(single):
        s = synth.opinions(g.n, "pareto", 950 + i)
        B.input(i).copy_(torch.from_numpy(s))
        ss.append(s)
    sm = np.stack([synth.opinions(multi.n, "pareto", 960 + q) for q in range(k)], axis=1)
    B.input(len(single)).copy_(torch.from_numpy(np.ascontiguousarray(sm)))
    stats, _ = B.solve()
    short = sum(1 for st in stats if not st["certified"])
    print(f"Pareto opinions: {short} item(s) short after the recorded budget", flush=True)
    assert B.check(extra_sweeps=1000) == 0
    _all_certified_against_oracle(B, single, multi, ss, sm, k)


def test_bound_caller_buffers_match_workspace_io():
    import paper_2507_14864_amd as fj
    single, multi = _items()
    k = 3
    B = fj.Batch([_dev(g) for g in single] + [_dev(multi)], [1] * len(single) + [k], eps=EPS, omega=1.4)
    ss, sm = _fill(B, single, multi, k)
    info = B.tune([1.2, 1.5])
    B.solve()
    z_io = [B.output(i).clone() for i in range(len(single) + 1)]
    s_user = [torch.from_numpy(s).to(DEV) for s in ss] + [torch.from_numpy(np.ascontiguousarray(sm)).to(DEV).view(-1)]
    z_user = [torch.full_like(t, -1.0) for t in s_user]
    B.bind(s_user, z_user)
    info_b = B.info()
    assert info_b["bound"] == 1 and info_b["graph_nodes"] == info["graph_nodes"] + 2
    for i in range(len(single) + 1):
        B.input(i).fill_(0.25)  # the bound inputs are copied over these at the solve's start
    for rep in range(2):
        stats, _ = B.solve()
        assert all(st["certified"] == 1 for st in stats)
        for i in range(len(single) + 1):
            assert torch.equal(z_user[i], z_io[i].reshape(-1)), (rep, i)
    B.bind()
    assert B.info()["bound"] == 0
    with pytest.raises(ValueError):
        B.bind(s_user[:-1], z_user[:-1])


def test_tuned_shape_is_reused_by_a_batch_of_the_same_shape():
    import paper_2507_14864_amd as fj
    fj.batch_tune_cache_clear()
    single, multi = _items()
    k = 3
    outs = []
    for trial in range(2):
        B = fj.Batch([_dev(g) for g in single] + [_dev(multi)], [1] * len(single) + [k], eps=EPS, omega=1.4)
        _fill(B, single, multi, k)
        info = B.tune([1.2, 1.5])
        assert info["cache_hit"] == trial, info
        assert info["union_chunks_in_flight"] in (2, 4, 8) and info["multi_arcs_in_flight"] in (4, 8, 16)
        stats, _ = B.solve()
        assert all(st["certified"] == 1 for st in stats)
        outs.append((info, [B.output(i).cpu().numpy().copy() for i in range(len(single) + 1)]))
        B.close()
    (i0, z0), (i1, z1) = outs
    for key in ("omega_undirected", "omega_directed", "omega_multi", "union_chunks_in_flight",
                "multi_arcs_in_flight", "sweep_budget"):
        assert i0[key] == i1[key], key
    for a, b in zip(z0, z1):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("weighted", [False, True])
def test_launch_parameters_leave_results_bit_identical(weighted):
    """Arcs in flight per wave (4, 8, 16) and 64-arc chunks per union tile
    (2, 4, 8) change only how the gathers are issued: the arc sums run in arc
    order with every setting, so the replays agree bit for bit.  Row lengths
    of the multi-vector graph (k = 64, and k = 5 with idle lanes) cover every
    remainder below 16 and rows above the light-row budget."""
    import paper_2507_14864_amd as fj
    single, _ = _items()
    multi = synth.chung_lu(20000, 150000, 2.1, 530, weighted=weighted)
    deg = np.diff(multi.row_ptr)
    assert set(range(1, 16)) <= set((deg % 16).tolist()) and deg.max() > 256
    for k in (64, 5):
        B = fj.Batch([_dev(g) for g in single] + [_dev(multi)], [1] * len(single) + [k], eps=EPS, omega=1.4)
        _fill(B, single, multi, k)
        B.tune([1.3, 1.5])
        ref = None
        for nch, mu in ((4, 8), (2, 4), (8, 16), (4, 16), (2, 8)):
            B.set_launch(nch, mu)
            assert (B.info()["union_chunks_in_flight"], B.info()["multi_arcs_in_flight"]) == (nch, mu)
            stats, mets = B.solve()
            out = [B.output(i).cpu().numpy().copy() for i in range(len(single) + 1)]
            assert all(s["certified"] == 1 for s in stats)
            if ref is None:
                ref = (out, [s["rounds"] for s in stats], mets)
                continue
            for i in range(len(out)):
                assert np.array_equal(out[i], ref[0][i]), (k, nch, mu, i)
            assert [s["rounds"] for s in stats] == ref[1]
            assert mets == ref[2]
        B.close()
    with pytest.raises(fj.FJError):
        B2 = fj.Batch([_dev(single[0])], [1], eps=EPS)
        B2.set_launch(3, 8)


def test_edge_visits_count_each_vector_until_quiet():
    """Per item, edge_visits counts the arcs gathered: a single-vector graph
    its sweeps times its arcs, a multi-vector item the sum over its vectors
    of the sweeps until each went quiet, times the arcs.  Two identical
    vectors go quiet together, at the item's last sweep; distinct ones add
    up to between the slowest alone and all of them at the last sweep."""
    import paper_2507_14864_amd as fj
    single, multi = _items()
    for same in (True, False):
        k = 2 if same else 4
        B = fj.Batch([_dev(g) for g in single] + [_dev(multi)], [1] * len(single) + [k], eps=EPS, omega=1.4)
        _fill(B, single, multi, k)
        if same:
            x = B.input(len(single))
            x[:, 1] = x[:, 0]
        stats, _ = B.solve()
        for i, g in enumerate(single):
            assert stats[i]["edge_visits"] == stats[i]["rounds"] * g.nnz
        st = stats[-1]
        assert st["certified"] == 1 and st["edge_visits"] % multi.nnz == 0
        per_vector = st["edge_visits"] // multi.nnz
        if same:
            assert per_vector == 2 * st["rounds"]
        else:
            assert st["rounds"] + (k - 1) <= per_vector <= k * st["rounds"]
        B.close()
