"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Sizes are small enough for the oracle to finish in seconds while spanning many
64-row tiles and a ragged last tile.  Tolerances follow from the method's
certificate: with c = sigma, eps' = eps/2 and every node with z >= sigma is
within relative error eps (Lemma 7 with Alg. 2's shift); the FP64 path is held
to 1e-6 relative on z and the measures, the FP32 path to 1e-4.
"""
import numpy as np
import pytest

import oracle
import synth
from tests import graphs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def fjmod():
    import paper_2507_14864_amd as fj
    return fj


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def check_solution(g, s, z_gpu, z_true, eps, c=1e-5, sigma=1e-5):
    """Entrywise bound of Lemma 7 after the shift, and the relative-error claim."""
    epsp = sigma * eps / (c + sigma)
    z = z_gpu.cpu().numpy()
    assert np.all(np.isfinite(z))
    bound = epsp * (z_true + c) * (1 + 1e-9) + 1e-15
    worst = np.max(np.abs(z - z_true) - bound)
    assert worst <= 0, f"Lemma 7 bound violated by {worst}"
    assert oracle.max_rel_error(z, z_true, floor=sigma) <= eps
    # the GPU certificate claim, recomputed by the oracle in FP64
    assert oracle.certificate(g, s, z, eps, sigma=sigma, c=c) <= 1.0 + 1e-9


# ------------------------------------------------------ config 1: BA n=2000
@pytest.mark.parametrize("schedule,omega", [("push", 1.0), ("sor", 1.0), ("sor", 1.5)])
def test_ba2000_fp64_against_dense(schedule, omega):
    fj = fjmod()
    g = synth.barabasi_albert(2000, 3, 1)
    s = synth.opinions(g.n, "uniform", 1)
    zt = oracle.dense_solve(g, s)
    G = fj.Graph.from_host(g, DEV, colour=True)
    sd = to_dev(s)
    z, st = fj.solve(G, sd, eps=1e-8, omega=omega, precision="fp64", schedule=schedule)
    assert st["certified"] == 1 and st["max_ratio"] <= 1.0
    check_solution(g, s, z, zt, 1e-8)
    m = fj.metrics(G, sd, z)
    mo = oracle.metrics(g, s, zt)
    for k in "PDIC":
        assert abs(m[k] - mo[k]) <= 1e-6 * abs(mo[k]), (k, m[k], mo[k])


# --------------------------------------------- FP32 path, mid-size power law
@pytest.mark.parametrize("directed", [False, True])
@pytest.mark.parametrize("schedule,omega", [("push", 1.0), ("sor", 1.0), ("sor", 1.3)])
def test_chung_lu_fp32_against_exact(directed, schedule, omega):
    fj = fjmod()
    n = 30011  # ragged last tile
    g = synth.chung_lu(n, 8 * n, 2.3 if not directed else 2.1, 7 + directed, directed=directed,
                       weighted=directed)
    s = synth.opinions(n, "bimodal", 8)
    zt = oracle.exact(g, s)
    G = fj.Graph.from_host(g, DEV, colour=True)
    sd = to_dev(s)
    z, st = fj.solve(G, sd, eps=1e-4, omega=omega, precision="fp32", schedule=schedule)
    assert st["certified"] == 1
    check_solution(g, s, z, zt, 1e-4)
    m = fj.metrics(G, sd, z)
    mo = oracle.metrics(g, s, zt)
    for k in "PDIC":
        assert abs(m[k] - mo[k]) <= 1e-4 * abs(mo[k]), (k, m[k], mo[k])


@pytest.mark.parametrize("kind", ["uniform", "exp", "pareto"])
def test_opinion_distributions(kind):
    """The paper's three opinion laws (Sec. 6); Pareto puts many s near 0,
    which the shift c must handle."""
    fj = fjmod()
    g = synth.chung_lu(20000, 100000, 2.3, 17)
    s = synth.opinions(g.n, kind, 18)
    zt = oracle.exact(g, s)
    G = fj.Graph.from_host(g, DEV, colour=True)
    for sched, omega in (("push", 1.0), ("sor", 1.5)):
        z, st = fj.solve(G, to_dev(s), eps=1e-4, omega=omega, schedule=sched)
        check_solution(g, s, z, zt, 1e-4)


# --------------------------------------------------------------- measures
def test_metrics_match_oracle_on_same_z_and_are_reproducible():
    fj = fjmod()
    for directed in (False, True):
        g = synth.chung_lu(50000, 300000, 2.2, 21, directed=directed, weighted=True)
        s = synth.opinions(g.n, "uniform", 22)
        z = synth.opinions(g.n, "beta", 23, a=2, b=2)  # any vector: the reductions are the unit under test
        G = fj.Graph.from_host(g, DEV)
        sd, zd = to_dev(s), to_dev(z)
        m1 = fj.metrics(G, sd, zd)
        m2 = fj.metrics(G, sd, zd)
        mo = oracle.metrics(g, s, z)
        for k in ("P", "D", "I", "C", "mean"):
            assert m1[k] == m2[k]  # bitwise: fixed-order reductions
            assert abs(m1[k] - mo[k]) <= 1e-12 * abs(mo[k]), (k, m1[k], mo[k])


@pytest.mark.parametrize("directed,weighted,schedule", [(False, False, "sor"), (False, True, "sor"),
                                                        (True, True, "sor"), (True, False, "push"),
                                                        (False, True, "push")])
def test_solve_measures_match_fj_metrics_and_oracle(directed, weighted, schedule):
    """fj_solve_opts.measures: on the SOR schedule D comes from the final
    certificate's gather pass (every stored arc, the differences of zhat',
    halved on an undirected graph), P/I/C/mean from the node passes on the
    returned z; other schedules run fj_metrics' passes.  P, I, C and the mean
    are the same kernels on the same z as fj_metrics, so bit for bit; D sums
    in another order, so within rounding; all against the oracle's measures of
    that z.  Heavy rows (over 256 arcs) are present, so the chunk waves add
    their arcs too."""
    fj = fjmod()
    g = synth.chung_lu(60000, 480000, 2.1, 951 + directed, directed=directed, weighted=weighted)
    assert np.diff(g.row_ptr).max() > 256
    s = synth.opinions(g.n, "bimodal", 953)
    G = fj.Graph.from_host(g, DEV, colour=schedule == "sor")
    sd = to_dev(s)
    z, st = fj.solve(G, sd, eps=1e-5, omega=1.0 if directed or schedule == "push" else 1.5, schedule=schedule,
                     measures=True)
    assert st["certified"] == 1
    m = st["measures"]
    ref = fj.metrics(G, sd, z)
    for k in ("P", "I", "C", "mean"):
        assert m[k] == ref[k], k
    assert abs(m["D"] - ref["D"]) <= 1e-12 * abs(ref["D"])
    mo = oracle.metrics(g, s, z.cpu().numpy())
    for k in ("P", "D", "I", "C", "mean"):
        assert abs(m[k] - mo[k]) <= 1e-12 * abs(mo[k]), (k, m[k], mo[k])
    # the same z and statistics as without the option
    z2, st2 = fj.solve(G, sd, eps=1e-5, omega=1.0 if directed or schedule == "push" else 1.5, schedule=schedule)
    assert torch.equal(z, z2) and st2["rounds"] == st["rounds"] and st2["max_ratio"] == st["max_ratio"]
    assert "measures" not in st2


def test_solve_measures_on_a_capped_solve():
    """A solve stopped by its work cap still returns the measures of its last
    estimate, with FJ_ERR_NOT_CONVERGED."""
    fj = fjmod()
    g = synth.chung_lu(20000, 160000, 2.3, 957)
    s = synth.opinions(g.n, "uniform", 958)
    G = fj.Graph.from_host(g, DEV, colour=True)
    with pytest.raises(fj.FJNotConverged) as e:
        fj.solve(G, to_dev(s), eps=1e-6, omega=1.5, schedule="sor", max_edge_visits=12 * (g.nnz + g.n),
                 measures=True)
    m = e.value.stats["measures"]
    ref = fj.metrics(G, to_dev(s), e.value.z)
    assert m["C"] == ref["C"] and abs(m["D"] - ref["D"]) <= 1e-12 * abs(ref["D"])


def test_certificate_matches_oracle():
    fj = fjmod()
    g = synth.chung_lu(40000, 200000, 2.3, 31, directed=True, weighted=True)
    s = synth.opinions(g.n, "uniform", 32)
    zt = oracle.exact(g, s)
    G = fj.Graph.from_host(g, DEV)
    for z in (zt * (1 + 2e-4), zt * (1 - 5e-5), s):
        want = oracle.certificate(g, s, z, 1e-4)
        got = fj.certify(G, to_dev(s), to_dev(z), 1e-4)
        assert abs(got - want) <= 1e-9 * max(1.0, want)
    # at the exact z the residual is FP64 rounding, whose value depends on the
    # order of the sums; both sides must only report it as far below 1
    assert oracle.certificate(g, s, zt, 1e-4) < 1e-3
    assert fj.certify(G, to_dev(s), to_dev(zt), 1e-4) < 1e-3


# ------------------------------------------------------------- edge cases
@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 127, 129])
def test_ragged_and_tiny(n):
    fj = fjmod()
    g = graphs.random_graph(n, min(1.0, 6.0 / max(n, 1)), 40 + n)
    s = synth.opinions(n, "uniform", 41)
    zt = oracle.dense_solve(g, s)
    G = fj.Graph.from_host(g, DEV, colour=True)
    for sched, omega in (("push", 1.0), ("sor", 1.7)):
        z, st = fj.solve(G, to_dev(s), eps=1e-6, omega=omega, precision="fp64", schedule=sched)
        check_solution(g, s, z, zt, 1e-6)


def test_graph_without_edges_returns_s():
    fj = fjmod()
    n = 1000
    g = synth.CSRGraph(n, np.zeros(n + 1, np.int32), np.zeros(0, np.int32), None, False)
    s = synth.opinions(n, "uniform", 5)
    G = fj.Graph.from_host(g, DEV, colour=True)
    for sched in ("push", "sor"):
        z, st = fj.solve(G, to_dev(s), eps=1e-6, precision="fp64", schedule=sched)
        assert np.allclose(z.cpu().numpy(), s, rtol=1e-6, atol=1e-11)


def test_constant_and_zero_opinions():
    fj = fjmod()
    g = synth.chung_lu(10000, 50000, 2.3, 51, directed=True, weighted=True)
    G = fj.Graph.from_host(g, DEV, colour=True)
    s = np.full(g.n, 0.42)
    for sched in ("push", "sor"):
        z, _ = fj.solve(G, to_dev(s), eps=1e-5, schedule=sched)
        assert np.allclose(z.cpu().numpy(), 0.42, rtol=1e-5)
    s0 = np.zeros(g.n)
    s0[::11] = 1.0
    zt = oracle.exact(g, s0)
    for sched in ("push", "sor"):
        z, _ = fj.solve(G, to_dev(s0), eps=1e-4, schedule=sched)
        check_solution(g, s0, z, zt, 1e-4)


def test_colouring_is_proper_and_classes_cover_nodes():
    fj = fjmod()
    for directed in (False, True):
        g = synth.chung_lu(30000, 200000, 2.1, 61, directed=directed)
        G = fj.Graph.from_host(g, DEV, colour=True)
        col = G.colours().cpu().numpy()
        rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
        assert np.all(col[rows] != col[g.col])  # no arc joins two nodes of one class
        sizes = G.colour_sizes()
        assert sum(sizes) == g.n and len(sizes) == col.max() + 1
        assert np.array_equal(np.bincount(col, minlength=len(sizes)), sizes)
        # first fit in some order (the colouring is first fit in priority
        # order): a node of colour c has neighbours (in A + A^T) of every
        # colour below c, whatever the order was
        src = np.concatenate([rows, g.col]).astype(np.int64)
        dst = np.concatenate([g.col, rows]).astype(np.int64)
        below = col[dst] < col[src]
        K = int(col.max()) + 1
        pairs = np.unique(src[below] * K + col[dst][below])
        have = np.bincount(pairs // K, minlength=g.n)
        assert np.array_equal(have, col), "a node skips a colour no neighbour holds"


def test_warm_start_reaches_same_certificate():
    fj = fjmod()
    g = synth.chung_lu(30000, 150000, 2.3, 71)
    s = synth.opinions(g.n, "bimodal", 72)
    zt = oracle.exact(g, s)
    G = fj.Graph.from_host(g, DEV, colour=True)
    sd = to_dev(s)
    for sched, omega in (("push", 1.0), ("sor", 1.4)):
        z_cold, st_cold = fj.solve(G, sd, eps=1e-4, omega=omega, schedule=sched)
        z_warm, st_warm = fj.solve(G, sd, eps=1e-4, omega=omega, schedule=sched, z0=to_dev(zt))
        assert st_warm["pushes"] == 0
        check_solution(g, s, z_warm, zt, 1e-4)
        z_s, st_s = fj.solve(G, sd, eps=1e-4, omega=omega, schedule=sched, z0=sd.clone())
        check_solution(g, s, z_s, zt, 1e-4)


# -------------------------------------------------------------- errors
def test_invalid_inputs_are_rejected():
    fj = fjmod()
    ok = graphs.from_arcs(4, [(0, 1), (1, 2), (2, 3)])
    bad_graphs = [
        synth.CSRGraph(3, np.array([0, 2, 2, 3], np.int32), np.array([2, 1, 0], np.int32), None, True),  # unsorted
        synth.CSRGraph(3, np.array([0, 1, 1, 1], np.int32), np.array([0], np.int32), None, True),  # self-loop
        synth.CSRGraph(3, np.array([0, 1, 1, 1], np.int32), np.array([7], np.int32), None, True),  # out of range
        synth.CSRGraph(3, np.array([0, 1, 1, 1], np.int32), np.array([1], np.int32), None, False),  # asymmetric
        synth.CSRGraph(3, np.array([0, 1, 1, 1], np.int32), np.array([1], np.int32),
                       np.array([-1.0], np.float32), True),  # negative weight
    ]
    for bg in bad_graphs:
        with pytest.raises(fj.FJError) as e:
            fj.Graph.from_host(bg, DEV)
        assert e.value.status == 1
    G = fj.Graph.from_host(ok, DEV, colour=True)
    with pytest.raises(fj.FJError) as e:
        fj.solve(G, to_dev(np.array([0.1, -0.2, 0.3, 0.4])), eps=1e-4)
    assert e.value.status == 1
    with pytest.raises(fj.FJError):
        fj.solve(G, to_dev(np.array([0.1, 0.2, 0.3, 0.4])), eps=1e-4, omega=1.5, schedule="push")
    with pytest.raises(fj.FJError):
        fj.solve(G, to_dev(np.array([0.1, 0.2, 0.3, 0.4])), eps=2.0)
    plain = fj.Graph.from_host(ok, DEV)
    with pytest.raises(fj.FJError):
        fj.solve(plain, to_dev(np.array([0.1, 0.2, 0.3, 0.4])), eps=1e-4, schedule="sor")


def test_work_cap_reports_not_converged():
    fj = fjmod()
    g = synth.chung_lu(20000, 100000, 2.3, 81)
    s = synth.opinions(g.n, "uniform", 82)
    G = fj.Graph.from_host(g, DEV, colour=True)
    for sched in ("push", "sor"):
        with pytest.raises(fj.FJNotConverged) as e:
            fj.solve(G, to_dev(s), eps=1e-6, schedule=sched, max_edge_visits=1000, check_every=1)
        assert e.value.stats["certified"] == 0
        assert np.all(np.isfinite(e.value.z.cpu().numpy()))


@pytest.mark.parametrize("directed", [False, True])
def test_sor_persistent_and_per_class_launches_agree(directed):
    """The persistent cooperative sweep and the one-launch-per-class sweep
    visit the colour classes in the same order, so both reach the certificate
    with the same number of sweeps and agree to rounding."""
    fj = fjmod()
    g = synth.chung_lu(60000, 600000, 2.2, 91 + directed, directed=directed, weighted=directed)
    s = synth.opinions(g.n, "bimodal", 92)
    zt = oracle.exact(g, s)
    G = fj.Graph.from_host(g, DEV, colour=True)
    sd = to_dev(s)
    omega = 1.6 if not directed else 1.2
    z1, st1 = fj.solve(G, sd, eps=1e-5, omega=omega, schedule="sor", persistent=True)
    z2, st2 = fj.solve(G, sd, eps=1e-5, omega=omega, schedule="sor", persistent=False)
    check_solution(g, s, z1, zt, 1e-5)
    check_solution(g, s, z2, zt, 1e-5)
    assert abs(st1["rounds"] - st2["rounds"]) <= 1
    assert np.max(np.abs(z1.cpu().numpy() - z2.cpu().numpy())) <= 1e-9


@pytest.mark.parametrize("directed,precision", [(False, "fp32"), (True, "fp32"), (False, "fp64")])
def test_sor_repeat_is_bitwise_identical(directed, precision):
    """Heavy rows are split into chunks whose partial sums are combined in
    fixed point, so the order in which chunks finish cannot change a bit of
    the result: two solves of the same problem return the same z and stats."""
    fj = fjmod()
    g = synth.chung_lu(200000, 4000000, 2.1, 95 + directed, directed=directed, weighted=directed)
    assert np.diff(g.row_ptr).max() > 4 * 256  # rows of several chunks
    s = synth.opinions(g.n, "bimodal", 96)
    G = fj.Graph.from_host(g, DEV, colour=True)
    sd = to_dev(s)
    omega = 1.6 if not directed else 1.2
    z1, st1 = fj.solve(G, sd, eps=1e-6, omega=omega, schedule="sor", precision=precision)
    z1 = z1.clone()
    z2, st2 = fj.solve(G, sd, eps=1e-6, omega=omega, schedule="sor", precision=precision)
    assert torch.equal(z1, z2)
    for key in ("rounds", "pushes", "certified"):
        assert st1[key] == st2[key], key
    check_solution(g, s, z2, oracle.exact(g, s), 1e-6)


def test_sor_star_beyond_packed_chunk_count():
    """A hub with more arcs than the one-launch sweep combines (4095 chunks of
    256) is swept by the two-launch path; its solution has a closed form:
    leaves satisfy 2 z_i - z_0 = s_i and the hub (1 + m) z_0 - sum z_i = s_0."""
    fj = fjmod()
    m = 4095 * 256 + 1000
    n = m + 1
    rp = np.zeros(n + 1, np.int64)
    rp[1] = m
    rp[2:] = m + np.arange(1, m + 1)
    col = np.empty(2 * m, np.int32)
    col[:m] = np.arange(1, n)
    col[m:] = 0
    g = synth.CSRGraph(n, rp.astype(np.int32), col, None, False)
    s = synth.opinions(n, "uniform", 97)
    z0 = (s[0] + 0.5 * s[1:].sum()) / (1.0 + 0.5 * m)
    zt = np.empty(n)
    zt[0] = z0
    zt[1:] = 0.5 * (s[1:] + z0)
    G = fj.Graph.from_host(g, DEV, colour=True)
    for precision in ("fp32", "fp64"):
        z, st = fj.solve(G, to_dev(s), eps=1e-6, omega=1.3, schedule="sor", precision=precision)
        assert st["certified"] == 1
        zz = z.cpu().numpy()
        assert np.max(np.abs(zz - zt) / (zt + 1e-5)) <= 1e-6


@pytest.mark.parametrize("directed", [False, True])
def test_stress_matches_oracle(directed):
    """Per-node stress (Sec. 3.4) and its total against the oracle on the same
    z, with heavy rows split into chunks; the total is reproducible bit for bit."""
    fj = fjmod()
    g = synth.chung_lu(20000, 200000, 2.1, 97 + directed, directed=directed, weighted=True)
    assert np.diff(g.row_ptr).max() > 256
    s = synth.opinions(g.n, "uniform", 98)
    z = synth.opinions(g.n, "beta", 99, a=2, b=2)
    G = fj.Graph.from_host(g, DEV)
    sd, zd = to_dev(s), to_dev(z)
    vec, total = fj.stress(G, sd, zd)
    _, total2 = fj.stress(G, sd, zd, per_node=False)
    want = oracle.stress(g, s, z)
    got = vec.cpu().numpy()
    assert np.all(np.abs(got - want) <= 1e-12 * np.abs(want) + 1e-300)
    assert total == total2
    assert abs(total - want.sum()) <= 1e-12 * want.sum()


@pytest.mark.parametrize("case", ["cycle", "complete", "star", "cl_undirected", "cl_directed"])
def test_estimate_omega_matches_spectral_radius(case):
    """Power iteration for mu = rho((I+D)^{-1} A) against closed forms and the
    oracle's eigenvalues; omega from Eq. (optimal-omega)."""
    fj = fjmod()
    if case == "cycle":
        g, mu = graphs.cycle(64), 2.0 / 3.0
    elif case == "complete":
        g, mu = graphs.complete(50), 49.0 / 50.0
    elif case == "star":
        g, mu = graphs.star(1000), np.sqrt(1000.0 / 2002.0)
    else:
        directed = case == "cl_directed"
        g = synth.chung_lu(1500, 9000, 2.2, 86 + directed, directed=directed, weighted=directed)
        mu = oracle.jacobi_spectral_radius(g)
    G = fj.Graph.from_host(g, DEV)
    r = fj.estimate_omega(G, max_iters=20000, tol=1e-12)
    assert abs(r["mu"] - mu) <= 2e-6 * mu, (r, mu)
    assert abs(r["omega"] - oracle.optimal_omega(r["mu"])) <= 1e-12


def test_tune_omega_keeps_fewest_updates():
    """The heuristic's choice is the candidate with the fewest updates, and
    its per-candidate counts are those of plain solves (deterministic)."""
    fj = fjmod()
    g = synth.chung_lu(30000, 240000, 2.3, 88)
    s = synth.opinions(g.n, "bimodal", 89)
    G = fj.Graph.from_host(g, DEV, colour=True)
    sd = to_dev(s)
    cands = [1.8, 1.6, 1.4, 1.2, 1.0]
    r = fj.tune_omega(G, sd, omegas=cands, eps=1e-5, schedule="sor")
    assert all(u > 0 for u in r["updates"])
    assert r["best"] == cands[int(np.argmin(r["updates"]))]
    for om, u in zip(cands[:2], r["updates"][:2]):
        _, st = fj.solve(G, sd, eps=1e-5, omega=om, schedule="sor")
        assert st["pushes"] == u


@pytest.mark.parametrize("gather_bits", [32, 64])
def test_gather_precision_reaches_the_same_certificate(gather_bits):
    """FP32 sweeps may start from the 32-bit fixed-point copy of the estimate
    or gather FP64 from the start; both end at the FP64 certificate."""
    fj = fjmod()
    n = 30011
    g = synth.chung_lu(n, 10 * n, 2.2, 101, weighted=True)
    s = synth.opinions(n, "bimodal", 102)
    zt = oracle.exact(g, s)
    G = fj.Graph.from_host(g, DEV, colour=True)
    z, st = fj.solve(G, to_dev(s), eps=1e-5, omega=1.5, schedule="sor", gather_bits=gather_bits)
    assert st["certified"] == 1
    check_solution(g, s, z, zt, 1e-5)
    assert (st["mirror_rounds"] > 0) == (gather_bits == 32)


@pytest.mark.parametrize("schedule", ["sor", "push"])
@pytest.mark.parametrize("scale", [1.0, 1.4, 3.0, 250.0])
def test_opinions_beyond_the_fixed_point_range(schedule, scale):
    """The 32-bit copy holds |zhat'| < 2, so it is used only while s' and
    the start stay below 1.5; larger opinions gather FP64 from the start.
    Either way the result meets the same bound, and scaling s scales z
    (the map s -> (I+L)^-1 s is linear, c scaled along)."""
    fj = fjmod()
    n = 20011
    g = synth.chung_lu(n, 8 * n, 2.3, 131)
    s = synth.opinions(n, "bimodal", 132) * scale
    zt = oracle.exact(g, s, tol=1e-12 * scale)  # the residual scales with s
    G = fj.Graph.from_host(g, DEV, colour=True)
    c = 1e-5 * scale
    z, st = fj.solve(G, to_dev(s), eps=1e-4, omega=1.0 if schedule == "push" else 1.5, schedule=schedule,
                     c=c, sigma=c)
    assert st["certified"] == 1
    check_solution(g, s, z, zt, 1e-4, c=c, sigma=c)
    assert (st["mirror_rounds"] > 0) == (scale * (1 + 1e-5) < 1.5)


@pytest.mark.parametrize("omega", [1.0, 1.6])
def test_merged_tail_reaches_the_same_certificate(omega):
    """The trailing small colour classes swept as one launch (a Jacobi step
    among their rows, allowed by the Householder-John bound) certify like the
    one-launch-per-class sweep, and the merged sweep is reproducible."""
    fj = fjmod()
    g = synth.chung_lu(200000, 2000000, 2.3, 103)
    s = synth.opinions(g.n, "bimodal", 104)
    zt = oracle.exact(g, s)
    G = fj.Graph.from_host(g, DEV, colour=True)
    sd = to_dev(s)
    z1, st1 = fj.solve(G, sd, eps=1e-5, omega=omega, schedule="sor")
    z1 = z1.clone()
    z2, st2 = fj.solve(G, sd, eps=1e-5, omega=omega, schedule="sor")
    z3, st3 = fj.solve(G, sd, eps=1e-5, omega=omega, schedule="sor", tail_merge=False)
    assert st1["merged_classes"] >= 2 and st3["merged_classes"] == 0
    assert torch.equal(z1, z2)
    for z, st in ((z1, st1), (z3, st3)):
        assert st["certified"] == 1
        check_solution(g, s, z, zt, 1e-5)


@pytest.mark.parametrize("directed", [False, True])
def test_push_rounds_gather_and_scatter_forms(directed):
    """The bulk push rounds in gather form (rows recompute their residual from
    the round's start) and in atomic scatter form (a node pushes whatever its
    residual holds when its wave reaches it, contributions of the same round
    included) both reach the certificate."""
    fj = fjmod()
    g = synth.chung_lu(40000, 400000, 2.2, 105 + directed, directed=directed, weighted=directed)
    s = synth.opinions(g.n, "uniform", 106)
    zt = oracle.exact(g, s)
    G = fj.Graph.from_host(g, DEV)
    sd = to_dev(s)
    zg, stg = fj.solve(G, sd, eps=1e-5, omega=1.0, schedule="push")
    zg = zg.clone()
    zs, sts = fj.solve(G, sd, eps=1e-5, omega=1.0, schedule="push", push_scatter=True)
    for z, st in ((zg, stg), (zs, sts)):
        assert st["certified"] == 1
        check_solution(g, s, z, zt, 1e-5)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_tiny_thresholds_at_hubs(precision):
    """Normalised Pareto opinions put many s near 0, so h = eps' (s + c) is
    about 5e-12 at eps = 1e-6 while hub rows sum thousands of arcs in chunks:
    the heavy-row combine must resolve far below that."""
    fj = fjmod()
    g = synth.chung_lu(300000, 3000000, 2.1, 107)
    assert np.diff(g.row_ptr).max() > 8 * 256
    s = synth.opinions(g.n, "pareto", 108)
    zt = oracle.exact(g, s)
    G = fj.Graph.from_host(g, DEV, colour=True)
    z, st = fj.solve(G, to_dev(s), eps=1e-6, omega=1.5, schedule="sor", precision=precision)
    assert st["certified"] == 1
    check_solution(g, s, z, zt, 1e-6)


@pytest.mark.parametrize("directed", [False, True])
def test_metric_bounds_match_oracle(directed):
    """A-posteriori bounds on the measures (Lemma 7 from the residual level)
    against the oracle on the same z, heavy rows included; the measures equal
    fj_metrics bit for bit, and a certified solve's bounds hold the exact
    measures."""
    fj = fjmod()
    c = 1e-5
    g = synth.chung_lu(20000, 120000, 2.2, 181 + directed, directed=directed, weighted=True)
    assert np.diff(g.row_ptr).max() > 256
    s = synth.opinions(g.n, "uniform", 183)
    zt = oracle.exact(g, s)
    G = fj.Graph.from_host(g, DEV, colour=True)
    sd = to_dev(s)
    rng = np.random.default_rng(184)
    for rel in (1e-8, 1e-6):
        z = zt * (1.0 + rel * rng.uniform(-1, 1, g.n))
        zd = to_dev(z)
        m, b, tau = fj.metrics_bounds(G, sd, zd, c=c)
        assert m == fj.metrics(G, sd, zd)
        bo, to = oracle.metrics_bounds(g, s, z, c)
        assert to < 1.0 and abs(tau - to) <= 1e-6 * to
        for k in ("P", "D", "I", "C", "mean"):
            assert abs(b[k] - bo[k]) <= 1e-6 * bo[k], (k, b[k], bo[k])
    _, b, tau = fj.metrics_bounds(G, sd, to_dev(np.full(g.n, 5.0)), c=c)
    assert tau >= 1.0 and all(np.isinf(v) for v in b.values())
    eps = 1e-4
    z, st = fj.solve(G, sd, eps=eps, omega=1.0 if directed else 1.5, schedule="sor")
    assert st["certified"] == 1
    m, b, tau = fj.metrics_bounds(G, sd, z, c=c)
    assert tau <= 1e-5 * eps / (c + 1e-5) * (1 + 1e-9)
    mt = oracle.metrics(g, s, zt)
    for k in ("P", "D", "I", "C", "mean"):
        assert abs(m[k] - mt[k]) <= b[k] + 1e-12 * abs(mt[k]), k


@pytest.mark.parametrize("n,check_every", [(3001, 1), (20011, 1), (20011, 3), (200000, 2)])
def test_grouped_skipping_launches_are_bit_exact(n, check_every):
    """Short batches switch to the launches with 8 light tiles per wave right
    after the first skipping sweep, so most of the late sweeps run grouped;
    small graphs leave ragged groups (fewer than 8 tiles at a class end).
    z, sweeps, updates and the certificate ratio equal those without
    skipping."""
    fj = fjmod()
    g = synth.chung_lu(n, 10 * n, 2.3, 211 + check_every)
    s = synth.opinions(g.n, "bimodal", 212)
    G = fj.Graph.from_host(g, DEV, colour=True)
    sd = to_dev(s)
    kw = dict(eps=1e-5, omega=1.6, schedule="sor", check_every=check_every)
    z0, st0 = fj.solve(G, sd, skip_below=-1.0, **kw)
    z1, st1 = fj.solve(G, sd, skip_below=0.2, **kw)
    assert st0["certified"] == 1 and st1["skipped_rows"] > 0
    assert torch.equal(z0, z1)
    assert (st1["rounds"], st1["pushes"], st1["max_ratio"]) == (st0["rounds"], st0["pushes"], st0["max_ratio"])
    assert st1["edge_visits"] + st1["skipped_arcs"] == st1["rounds"] * g.nnz


@pytest.mark.parametrize("directed,weighted,precision,gather_bits,omega",
                         [(False, False, "fp32", 0, 1.6), (True, True, "fp32", 0, 1.0), (False, True, "fp32", 0, 1.6),
                          (False, False, "fp64", 0, 1.6), (False, False, "fp32", 64, 1.6),
                          (True, True, "fp32", 0, 1.2), (True, False, "fp64", 0, 1.1), (True, True, "fp32", 64, 1.1)])
def test_bound_skipping_is_bit_exact(directed, weighted, precision, gather_bits, omega):
    """A row is skipped only while its residual bound (its own residual at its
    last sweep, raised by a_ij |change| for every later update of a node it
    reads, Lemma 4) plus its gather rounding stays below the threshold, so it
    would not have updated: the same z bit for bit, the same sweeps and
    updates, with and without skipping (bounds from the second sweep and
    skipping from the third with skip_below = 1, and at the default fraction
    0.05 set explicitly, since by default a graph of under 2^24 arcs does not
    skip); merged tail included.  On directed graphs the rows to raise come from the
    relabelled CSR(A^T), so a slip there (a missing or misweighted reader)
    would let a row skip an update and change z."""
    fj = fjmod()
    g = synth.chung_lu(200000, 2000000, 2.3, 191 + directed, directed=directed, weighted=weighted)
    s = synth.opinions(g.n, "bimodal", 192)
    G = fj.Graph.from_host(g, DEV, colour=True)
    sd = to_dev(s)
    kw = dict(eps=1e-5, omega=omega, schedule="sor", precision=precision, gather_bits=gather_bits)
    z0, st0 = fj.solve(G, sd, skip_below=-1.0, **kw)
    assert st0["certified"] == 1 and st0["skipped_rows"] == 0
    # rows of more than 256 arcs gather FP64 in every fixed-point sweep
    deg = np.diff(g.row_ptr)
    heavy_arcs = int(deg[deg > 256].sum())
    assert heavy_arcs > 0
    assert st0["mirror_fp64_edge_visits"] == st0["mirror_rounds"] * heavy_arcs
    zd, std = fj.solve(G, sd, **kw)  # the default: no skipping at this size
    assert g.nnz < 1 << 24 and std["skipped_rows"] == 0 and torch.equal(z0, zd)
    for below in (1.0, 0.05):
        z1, st1 = fj.solve(G, sd, skip_below=below, **kw)
        assert torch.equal(z0, z1), below
        assert (st1["rounds"], st1["pushes"], st1["max_ratio"]) == (st0["rounds"], st0["pushes"], st0["max_ratio"])
        if below == 1.0:
            assert st1["skipped_rows"] > 0 and st1["bound_adds"] > 0
        # arcs gathered plus arcs of skipped rows cover every sweep
        assert st1["edge_visits"] + st1["skipped_arcs"] == st1["rounds"] * g.nnz
        assert 0 <= st1["mirror_edge_visits"] <= st1["mirror_rounds"] * g.nnz
        assert 0 <= st1["mirror_fp64_edge_visits"] <= min(st1["mirror_edge_visits"], st1["mirror_rounds"] * heavy_arcs)


def test_refinement_reseeds_from_the_fp64_residual():
    """FP32 push rounds (scatter form) at eps = 1e-7: the threshold
    eps' (s + c) lies below the FP32 rounding of the residual itself, so the
    rounds go quiet on an FP32 residual whose FP64 recomputation fails the
    certificate of Lemma 7.  The solve then re-seeds r from the FP64 residual
    and resumes until the certificate holds; the result meets Lemma 7's
    bound against the exact z."""
    fj = fjmod()
    g = synth.chung_lu(50000, 400000, 2.3, 961)
    s = synth.opinions(g.n, "uniform", 962)
    zt = oracle.exact(g, s)
    G = fj.Graph.from_host(g, DEV)
    z, st = fj.solve(G, to_dev(s), eps=1e-7, omega=1.0, precision="fp32", schedule="push", push_scatter=True)
    print(f"refinement: {st}", flush=True)
    assert st["refinements"] >= 1 and st["certified"] == 1 and st["max_ratio"] <= 1.0
    check_solution(g, s, z, zt, 1e-7)


def test_gather_probe_reports_a_rate():
    """fj_gather_probe times the sweep's index stream alone; bad sizes are rejected."""
    fj = fjmod()
    g = synth.chung_lu(50_000, 400_000, 2.3, 7)
    for colour in (True, False):
        G = fj.Graph.from_host(g, DEV, colour=colour)
        r4 = fj.gather_probe(G, 4, 3)
        r8 = fj.gather_probe(G, 8, 3)
        assert r4 > 0 and r8 > 0
        with pytest.raises(fj.FJError):
            fj.gather_probe(G, 2, 1)
        with pytest.raises(fj.FJError):
            fj.gather_probe(G, 4, 0)


@pytest.mark.parametrize("directed,precision,omega", [(False, "fp32", 1.0), (True, "fp32", 1.0), (False, "fp64", 1.0),
                                                      (True, "fp32", 0.8), (False, "fp64", 0.7)])
def test_frontier_push_rounds(directed, precision, omega):
    """Push rounds over the frontier queue (Alg. 1's queue as the round sets of
    the proof of Thm. 5) reach the certificate; omega < 1 exercises the nodes
    that queue themselves again.  Its pushes are the scan form's: the same
    certificate from a similar number of updates."""
    fj = fjmod()
    g = synth.chung_lu(40000, 400000, 2.2, 111 + directed, directed=directed, weighted=directed)
    s = synth.opinions(g.n, "bimodal", 112)
    zt = oracle.exact(g, s)
    G = fj.Graph.from_host(g, DEV)
    sd = to_dev(s)
    eps = 1e-6 if precision == "fp64" else 1e-5
    zf, stf = fj.solve(G, sd, eps=eps, omega=omega, schedule="push", precision=precision, push_scatter="frontier")
    zf = zf.clone()
    zs, sts = fj.solve(G, sd, eps=eps, omega=omega, schedule="push", precision=precision, push_scatter=True)
    print(f"frontier {stf['rounds']} rounds ({stf['mirror_rounds']} over the queue) {stf['pushes']} pushes; "
          f"scan {sts['rounds']} rounds {sts['pushes']} pushes", flush=True)
    assert stf["mirror_rounds"] > 0  # the sparse rounds popped the queue
    for z, st in ((zf, stf), (zs, sts)):
        assert st["certified"] == 1
        check_solution(g, s, z, zt, eps)
    assert stf["pushes"] <= 2 * sts["pushes"]


def test_frontier_hubs_refinement_and_warm_start():
    """Nodes with more than 2048 arcs to scatter take the block-per-node
    bucket; an FP32 residual at eps = 1e-7 forces refinements, which re-seed
    the frontier from the FP64 residual; a warm start seeds it from the start's
    residual (Lemma 4)."""
    fj = fjmod()
    g = synth.chung_lu(300000, 3000000, 2.1, 113)
    assert np.diff(g.row_ptr).max() > 2048
    s = synth.opinions(g.n, "uniform", 114)
    zt = oracle.exact(g, s)
    G = fj.Graph.from_host(g, DEV)
    sd = to_dev(s)
    z, st = fj.solve(G, sd, eps=1e-7, omega=1.0, precision="fp32", schedule="push", push_scatter="frontier")
    print(f"frontier refinement: {st}", flush=True)
    assert st["refinements"] >= 1 and st["certified"] == 1
    check_solution(g, s, z, zt, 1e-7)
    z2, st2 = fj.solve(G, sd, eps=1e-5, omega=1.0, schedule="push", push_scatter="frontier", z0=sd)
    assert st2["certified"] == 1
    check_solution(g, s, z2, zt, 1e-5)
    # an empty frontier from the exact solution: no push at all
    z3, st3 = fj.solve(G, sd, eps=1e-5, omega=1.0, precision="fp64", schedule="push", push_scatter="frontier",
                       z0=to_dev(zt))
    assert st3["certified"] == 1 and st3["pushes"] == 0


@pytest.mark.parametrize("form", [True, "frontier"])
def test_fp32_scatter_refinements_terminate(form):
    """Repeated FP32 scatter solves (run-dependent order) on a directed
    weighted graph of the 1M-node law: each ends certified after a few
    refinements.  A refinement re-seeds the residual rounded away from zero,
    so a row that fails the FP64 certificate by less than half an ulp of its
    FP32 threshold is still pushed."""
    fj = fjmod()
    g = synth.chung_lu(200_000, 2_000_000, 2.1, 121, directed=True, weighted=True)
    s = synth.opinions(g.n, "uniform", 122)
    zt = oracle.exact(g, s)
    G = fj.Graph.from_host(g, DEV)
    sd = to_dev(s)
    for rep in range(6):
        z, st = fj.solve(G, sd, eps=1e-4, omega=1.0, precision="fp32", schedule="push", push_scatter=form)
        assert st["certified"] == 1 and st["refinements"] <= 3, (rep, st)
        if rep == 0:
            check_solution(g, s, z, zt, 1e-4)


def test_fj_trace_writes_one_line_per_check(tmp_path):
    """FJ_TRACE=1: the solve writes JSON lines per batch of sweeps and per
    certificate to stderr, with nondecreasing cumulative counts, ending in a
    certificate without violations."""
    import json
    import os
    import subprocess
    import sys
    script = tmp_path / "trace_run.py"
    script.write_text(
        "import sys\n"
        f"sys.path.insert(0, {os.path.dirname(os.path.dirname(os.path.abspath(__file__)))!r})\n"
        "import torch, synth\n"
        "import paper_2507_14864_amd as fj\n"
        "g = synth.chung_lu(30000, 200000, 2.3, 131)\n"
        "s = torch.from_numpy(synth.opinions(g.n, 'uniform', 132)).to('cuda:0')\n"
        "G = fj.Graph.from_host(g, 'cuda:0', colour=True)\n"
        "z, st = fj.solve(G, s, eps=1e-5, omega=1.5, schedule='sor')\n"
        "z, st = fj.solve(G, s, eps=1e-5, omega=1.0, schedule='push', push_scatter='frontier')\n"
        "print('done', flush=True)\n")
    env = dict(os.environ, FJ_TRACE="1")
    out = subprocess.run([sys.executable, str(script)], env=env, capture_output=True, text=True, timeout=180)
    assert out.returncode == 0, out.stderr[-2000:]
    lines = [json.loads(l) for l in out.stderr.splitlines() if l.startswith("{\"fj_trace\"")]
    for sched in ("sor", "push"):
        ev = [l for l in lines if l["fj_trace"] == sched]
        batches = [l for l in ev if l["event"] == "batch"]
        certs = [l for l in ev if l["event"] == "certificate"]
        assert batches and certs, sched
        ups = [b["updates"] for b in batches]
        assert ups == sorted(ups) and batches[-1]["rounds"] >= batches[0]["rounds"]
        assert certs[-1]["violations"] == 0 and certs[-1]["max_ratio"] <= 1.0


@pytest.mark.parametrize("omega", [1.5, 1.8])
def test_directed_over_relaxation_fails_alike_in_oracle_and_gpu(omega):
    """On a directed graph of the 1M-node law (out/in exponent 2.1, weights
    U[0.5, 1.5]) at 100k nodes, over-relaxation beyond 1.2 is outside what
    Sec. 5.2 argues (symmetric I+L).  The oracle's FIFO push and the GPU's
    colour-ordered sweeps are pinned to fail alike: neither certifies within
    its work cap (the oracle may also report divergence), and the GPU reports
    it with FJ_ERR_NOT_CONVERGED and a finite estimate instead of a wrong
    certificate."""
    fj = fjmod()
    g = synth.chung_lu(100_000, 1_000_000, 2.1, 141, directed=True, weighted=True)
    s = synth.opinions(g.n, "uniform", 142)
    cap = 200 * (g.nnz + g.n)
    p = oracle.push(g, s, 1e-4, omega=omega, max_edge_visits=cap)
    print(f"omega {omega}: oracle capped {p['capped']} diverged {p['diverged']}", flush=True)
    assert p["capped"] or p["diverged"]
    G = fj.Graph.from_host(g, DEV, colour=True)
    with pytest.raises(fj.FJNotConverged) as e:
        fj.solve(G, to_dev(s), eps=1e-4, omega=omega, schedule="sor", max_edge_visits=cap)
    assert e.value.stats["certified"] == 0
    print(f"omega {omega}: GPU {e.value.stats['rounds']} sweeps, max ratio {e.value.stats['max_ratio']}", flush=True)
