#!/usr/bin/env python3
"""Benchmark: time to a certified relative error of 1e-4 for the FJ equilibrium
of a 10M-node undirected power-law graph on one MI355X, plus the Table 1
measures.

One step = the whole hot path over the resident synthetic input: shift and
init (Alg. 2), over-relaxed sweeps or push rounds (Alg. 1/3), FP64
certificate, unshift, and the P/D/I/C reductions.  Graph ingest (validation,
degrees, colouring, relabelling) happens once before the timed region and is
reported separately.

Prints one JSON line (rank 0).  Diagnostics go to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
HERE = ROOT
sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: (n, edge samples, gamma, directed, weighted, seed, opinion kind, eps, default omega)
    "cl10m": dict(n=10_000_000, m=100_000_000, gamma=2.3, directed=False, weighted=False, seed=3,
                  s_kind="bimodal", eps=1e-4, omega=1.6,
                  desc="undirected Chung-Lu n=10M, 100M edge samples (~200M stored arcs), gamma=2.3, "
                       "unit weights, s=0.5Beta(2,8)+0.5Beta(8,2)"),
    "cl1m_directed": dict(n=1_000_000, m=10_000_000, gamma=2.1, directed=True, weighted=True, seed=2,
                          s_kind="uniform", eps=1e-4, omega=1.0,
                          desc="directed Chung-Lu n=1M, 10M arcs, out/in exponent 2.1, weights U[0.5,1.5], "
                               "s~U[0,1]"),
    "ba2000": dict(n=2000, m=3, gamma=0.0, directed=False, weighted=False, seed=1, s_kind="uniform", eps=1e-8,
                   omega=1.0, desc="Barabasi-Albert n=2000 m=3, s~U[0,1], FP64"),
}

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_input(wl):
    import synth
    if wl["gamma"] == 0.0:
        g = synth.barabasi_albert(wl["n"], wl["m"], wl["seed"])
    else:
        g = synth.chung_lu(wl["n"], wl["m"], wl["gamma"], wl["seed"], directed=wl["directed"],
                           weighted=wl["weighted"])
    s = synth.opinions(g.n, wl["s_kind"], wl["seed"])
    return g, s


def algorithmic_bytes(schedule, stats, n, nnz, weighted, gather_rounds=False, frontier=False):
    """Bytes the iteration kernel must move, without cache reuse.

    Colour-class sweep (pull form): per row scanned 28 B (row_ptr 4, s' 8,
    1+d 8, own zhat' 8); per updated row 20 B (1/(1+d) 8, zhat' write 8,
    fixed-point copy write 4); per arc 4 B column index plus the gathered
    value, 8 B (FP64) or 4 B in the sweeps that gather the fixed-point copy,
    where rows of more than 256 arcs still gather 8 B (light rows the copy
    cannot resolve also do, and are counted at 4 B, so the figure is low by
    those); +4 B per arc with weights.  A row skipped by its residual bound counts
    its row data and the bound (28 + 8 B) and none of its arcs; keeping the
    bounds (a write per swept row, an atomic add per arc of an updated row)
    is not counted.
    Push round: per node scanned 8 B (r, h), per push 44 B (row_ptr 8, r
    exchange 8, 1/(1+d) 4+8, zhat' RMW 16), per arc 12 B (col 4 + residual
    atomic RMW 8), +4 B with weights.  Over a frontier queue no node is
    scanned; a popped node reads its queue entry, clears its queue flag and
    reads r and h (16 B), counted per push."""
    if schedule == "sor" or gather_rounds:
        arcs = stats["edge_visits"]
        mirror_arcs = stats["mirror_edge_visits"] if schedule == "sor" else stats.get("mirror_rounds", 0) * nnz
        mirror_fp64 = stats.get("mirror_fp64_edge_visits", 0) if schedule == "sor" else 0
        gather = 8 * (arcs - mirror_arcs) + 4 * (mirror_arcs - mirror_fp64) + 8 * mirror_fp64
        skipped = stats.get("skipped_rows", 0)
        return (28 * stats["rounds"] * n + 8 * skipped + 20 * stats["pushes"] + 4 * arcs + gather
                + (4 * arcs if weighted else 0))
    per_arc = 16 if weighted else 12
    if frontier:
        return 60 * stats["pushes"] + per_arc * stats["edge_visits"]
    return 8 * stats["rounds"] * n + 44 * stats["pushes"] + per_arc * stats["edge_visits"]


KERNEL_SOURCES = ("fj_sor.h", "fj_tile.h", "fj_device.h")
TRAFFIC_FILE = os.path.join(HERE, "profiles", "k_sor_class_cl10m_pmc.txt")


def kernel_sources_hash():
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(HERE, "paper_2507_14864_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM-side bytes per launch of the sweep kernel from the committed
    FETCH_SIZE/WRITE_SIZE counter summary, or None when the kernel sources
    changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            fields = dict(line.split(":", 1) for line in f if ":" in line)
    except OSError:
        return None
    if fields.get("kernel_sources_sha256", "").strip() != kernel_sources_hash():
        return None
    try:
        return int(float(fields["traffic_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def host_cpu_model():
    """The host CPU's model name (first processor in /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(wl, g, s, gpu_edge_visits=None):
    """The oracle's sequential ImprovedBLISOR (FIFO, FP64, one core) on the
    same input the GPU solves, to the same eps with the same omega (omega 1
    on directed graphs).  Beside it, the oracle's exact solve of that input
    (PCG on all host threads, or sequential Gauss-Seidel when directed, to a
    residual of 1e-12), whose z is returned for the error report, and the
    ratio of the GPU's edge visits to the sequential push's (the work
    efficiency of the parallel schedule)."""
    import oracle
    omega = wl["omega"] if not wl["directed"] else 1.0
    t0 = time.perf_counter()
    p = oracle.push(g, s, wl["eps"], omega=omega)
    dt = time.perf_counter() - t0
    out = dict(value=round(dt, 3), unit="s", cores=1, kind="oracle",
               sample=f"sequential FIFO ImprovedBLISOR (omega={omega}, eps={wl['eps']}, FP64) fully solved on the "
                      f"benchmark's own input ({g.n} nodes, {g.nnz} arcs; {p['edge_visits']} edge visits)",
               host_cpu=host_cpu_model(), host_threads=os.cpu_count())
    if gpu_edge_visits is not None:
        out["gpu_to_oracle_edge_visits"] = round(gpu_edge_visits / max(p["edge_visits"], 1), 3)
    t0 = time.perf_counter()
    zt = oracle.exact(g, s)
    out["exact_solve"] = {"value": round(time.perf_counter() - t0, 2), "unit": "s",
                          "cores": 1 if g.directed else oracle.threads(),
                          "kind": "oracle Gauss-Seidel" if g.directed else "oracle Jacobi-PCG",
                          "sample": "the full input, to ||s - (I+L) z||_inf <= 1e-12"}
    return out, zt, p["z"]


def errors_vs_exact(g, s, z, zt, eps):
    """Measured errors of a solve against the oracle's exact z: the largest
    relative error of z where z_exact >= sigma = 1e-5 (the ImprovedBLI
    guarantee), and the relative error of each Table 1 measure."""
    import oracle
    m, mt = oracle.metrics(g, s, z), oracle.metrics(g, s, zt)
    return {"z_max_rel": float(f"{oracle.max_rel_error(z, zt, floor=1e-5):.3e}"),
            **{k: float(f"{abs(m[k] - mt[k]) / abs(mt[k]):.3e}") for k in "PDIC"}, "eps": eps}


# The network's two MFMA tile kernels, per node.  Flops: the products of the
# layers (layer 1: 8 x 64 and P = H1 Wp, 64 x 16; k_net_l2: layer 1 again,
# [H1 | M] W2, 80 x 64, and the readout u, 64), 2 per multiply-add.  Bytes:
# s 8, 1 + d 8, the FP32 neighbour sum of s 4, then P written (16 BF16, 32)
# or M read (32) and z0 written (8).
NET_L1 = {"flop": 2 * (8 * 64 + 64 * 16), "bytes": 8 + 8 + 4 + 32}
NET_L2 = {"flop": 2 * (8 * 64 + 80 * 64 + 64), "bytes": 8 + 8 + 4 + 32 + 8}
MFMA_BF16_TFLOPS = 2500.0


def dense_layer_roofline(G, sd, params, reps=7):
    """Median stage times of the forward (HIP events) and the two MFMA tile
    kernels against the bf16 dense MFMA peak and the HBM peak."""
    import paper_2507_14864_amd as fj
    runs = [fj.wsnet_forward_timed(G, sd, params)[1] for _ in range(reps)]
    med = [sorted(r[q] for r in runs)[reps // 2] for q in range(4)]
    n = G.n
    out = {"stage_ms": {"gather_s": round(med[0], 4), "k_net_l1": round(med[1], 4), "gather_P": round(med[2], 4),
                        "k_net_l2": round(med[3], 4)}}
    for name, ms, spec in (("k_net_l1", med[1], NET_L1), ("k_net_l2", med[3], NET_L2)):
        tf = spec["flop"] * n / (ms * 1e-3) / 1e12
        gb = spec["bytes"] * n / (ms * 1e-3) / 1e9
        out[name] = {"flop_per_node": spec["flop"], "bytes_per_node": spec["bytes"], "tflops": round(tf, 1),
                     "mfma_frac": round(tf / MFMA_BF16_TFLOPS, 4), "gbs": round(gb, 1),
                     "hbm_frac": round(gb / HBM_PEAK_GBS, 4)}
    return out


def warm_start_eval(dev):
    """Warm vs cold start on the held-out directed graph (5M nodes, 50M arc
    samples, bimodal opinions) with the stored network weights: time to the
    same certificate (eps 1e-4, omega 1.1), inference included, beside the
    untrained controls z0 = s and z0 = k FJ steps (Eq. (1))."""
    import torch
    import paper_2507_14864_amd as fj
    from paper_2507_14864_amd import warmstart
    params = warmstart.load_params(dev)
    if params is None:
        return None
    g, s = warmstart.heldout_problem()
    G = fj.Graph.from_host(g, dev, colour=True)
    sd = torch.from_numpy(s).to(dev)
    res = warmstart.evaluate(G, sd, params, eps=1e-4, omega=1.1, jacobi=(2, 4))
    out = {"workload": "directed Chung-Lu n=5M, 50M arc samples, exponent 2.1, weights U[0.5,1.5], bimodal s",
           "omega": 1.1, "cold_s": round(res["cold"]["s"], 5), "net_s": round(res["net"]["s"], 5),
           "net_inference_s": round(res["net"]["inference_s"], 5),
           "sweeps": {k: v["sweeps"] for k, v in res.items() if isinstance(v, dict)},
           "speedup_vs_cold": round(res["speedup_net_vs_cold"], 3),
           "speedup_vs_best_untrained_control": round(res["speedup_net_vs_best_control"], 3),
           "controls_s": {k: round(v["s"], 5) for k, v in res.items() if k.startswith("z0=")},
           "dense_layers": dense_layer_roofline(G, sd, params)}
    del G
    torch.cuda.empty_cache()
    return out


def batch_inputs():
    """64 vectors (22 U[0,1], 21 Beta(2,2), 21 bimodal; seeds 400-463) on an
    undirected Chung-Lu graph with 2M nodes and 20M edge samples (gamma 2.3,
    seed 4), plus 256 graphs with log-uniform sizes in [1k, 200k] and average
    degree 8, alternately undirected (unit weights) and directed with
    U[0.5,1.5] weights (seeds 500-755), each with one U[0,1] vector."""
    import numpy as np
    import synth
    big = synth.chung_lu(2_000_000, 20_000_000, 2.3, 4)
    S = []
    for q in range(64):
        kind = "uniform" if q < 22 else ("beta" if q < 43 else "bimodal")
        S.append(synth.opinions(big.n, kind, 400 + q, a=2, b=2) if kind == "beta"
                 else synth.opinions(big.n, kind, 400 + q))
    S = np.ascontiguousarray(np.stack(S, axis=1))
    rng = np.random.default_rng(12345)
    smalls, ss = [], []
    for i in range(256):
        n = int(round(np.exp(rng.uniform(np.log(1000), np.log(200000)))))
        directed = (i % 2 == 1)
        m = 8 * n if directed else 4 * n
        smalls.append(synth.chung_lu(n, m, 2.1 if directed else 2.3, 500 + i, directed=directed,
                                     weighted=directed))
        ss.append(synth.opinions(n, "uniform", 500 + i))
    return big, S, smalls, ss


def batch_eval(dev, steps, warmup):
    """The batched solve (64 vectors on the 2M-node graph plus 256 graphs of
    1k-200k nodes): ingest, tune, then `steps` replays of the recorded
    sequence timed between device synchronizations."""
    import torch
    import paper_2507_14864_amd as fj
    t0 = time.perf_counter()
    big, S, smalls, ss = batch_inputs()
    log(f"batch inputs generated in {time.perf_counter() - t0:.1f}s: big n={big.n} nnz={big.nnz}, "
        f"{len(smalls)} graphs with {sum(g.n for g in smalls)} nodes / {sum(g.nnz for g in smalls)} arcs")

    def dev_graph(g):
        return (torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col).to(dev),
                None if g.w is None else torch.from_numpy(g.w).to(dev), g.directed)

    t0 = time.perf_counter()
    B = fj.Batch([dev_graph(big)] + [dev_graph(g) for g in smalls], [64] + [1] * len(smalls), eps=1e-4,
                 omega=1.5)
    B.input(0).copy_(torch.from_numpy(S))
    for i, s in enumerate(ss):
        B.input(i + 1).copy_(torch.from_numpy(s))
    torch.cuda.synchronize()
    ingest = time.perf_counter() - t0
    t0 = time.perf_counter()
    info = B.tune([1.2, 1.4, 1.5, 1.6, 1.7])
    tune_s = time.perf_counter() - t0
    log(f"batch ingest {ingest:.2f}s, tune {tune_s:.2f}s: {info}")
    for _ in range(warmup):
        B.solve_async()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        B.solve_async()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / max(steps, 1)
    stats, mets = B.results()
    cert = sum(s["certified"] for s in stats)
    # gathered value bytes: 8 per arc and vector swept (a lower bound on the
    # traffic: column indices, row data and writes come on top)
    gathered = 8 * sum(s["edge_visits"] for s in stats)
    # all algorithmic bytes, as for the single solve: the multi-vector item per
    # vector and row swept 24 (s' and zhat' read, zhat' written) and per arc
    # and vector 8 (the gathered value), and per arc and sweep 4 (the column
    # index, read once per row for all vectors); a single-vector graph per row
    # and sweep 36 (row offset 4, s' 8, 1 + d 8, zhat' read and written 16) and
    # per arc and sweep 12 (+4 with weights)
    vec_sweeps = stats[0]["edge_visits"] / max(big.nnz, 1)
    algorithmic = (24 * big.n * vec_sweeps + 8 * stats[0]["edge_visits"] + 4 * big.nnz * stats[0]["rounds"])
    for g, st in zip(smalls, stats[1:]):
        algorithmic += 36 * g.n * st["rounds"] + (16 if g.w is not None else 12) * st["edge_visits"]
    out = {"workload": "64 vectors (U[0,1], Beta(2,2), bimodal) on an undirected Chung-Lu graph with 2M nodes / "
                       "20M edge samples, plus 256 graphs of 1k-200k nodes (average degree 8, half directed)",
           "s_per_batch": round(dt, 5), "vector_solves_per_s": round(320 / dt, 1), "eps": 1e-4,
           "omega_multi": info["omega_multi"], "omega_undirected": info["omega_undirected"],
           "omega_directed": info["omega_directed"], "sweep_budget": info["sweep_budget"],
           "graph_nodes": info["graph_nodes"], "union_chunks_in_flight": info["union_chunks_in_flight"],
           "multi_arcs_in_flight": info["multi_arcs_in_flight"], "certified_items": cert, "items": len(stats),
           "max_sweeps_used": max(s["rounds"] for s in stats),
           "gathered_value_bytes": gathered, "gathered_GBs": round(gathered / dt / 1e9, 1),
           "gathered_hbm_frac": round(gathered / dt / 1e9 / HBM_PEAK_GBS, 4),
           "algorithmic_bytes": int(algorithmic), "algorithmic_GBs": round(algorithmic / dt / 1e9, 1),
           "algorithmic_hbm_frac": round(algorithmic / dt / 1e9 / HBM_PEAK_GBS, 4), "ingest_s": round(ingest, 2),
           "tune_s": round(tune_s, 2), "steps": steps}
    B.close()  # release the recorded hipGraph while the runtime is up
    del B
    torch.cuda.empty_cache()
    return out


def bench_batch(args):
    out = batch_eval("cuda:0", args.steps, args.warmup)
    dt = out["s_per_batch"]
    line = {
        "metric": "batched FJ solve time (64 vectors on a 2M-node graph + 256 graphs of 1k-200k nodes, eps 1e-4)",
        "value": dt, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(dt * 1000, 3), "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic", "config": {"workload": "batch", **out},
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cl10m", choices=sorted(WORKLOADS) + ["batch"])
    ap.add_argument("--schedule", default="sor", choices=["sor", "push"])
    ap.add_argument("--opinions", default=None, choices=["uniform", "exp", "pareto", "bimodal"],
                    help="override the workload's opinion law (the paper's three laws of Sec. 6, or bimodal)")
    ap.add_argument("--omega", default=None,
                    help="a number, 'young' (Eq. (optimal-omega) from a power-iteration estimate of mu) or "
                         "'tune' (the paper's heuristic: fewest updates over 1.95, 1.90, ..., 1.0); "
                         "the estimate or the tuning runs before the timed steps")
    ap.add_argument("--precision", default=None, choices=["fp32", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-warm-start", action="store_true",
                    help="skip the learned warm start evaluation on the held-out 5M-node directed graph")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched solve (64 vectors on a 2M-node graph + 256 small graphs)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 512 MiB device copy (counter calibration under rocprofv3)")
    ap.add_argument("--gather-bits", type=int, default=0, choices=[0, 32, 64],
                    help="FP32 sweeps: gather the 32-bit fixed-point copy first (0, 32) or FP64 from the start (64)")
    ap.add_argument("--push-frontier", action="store_true",
                    help="push rounds over a frontier queue (atomic scatter of the popped nodes only)")
    ap.add_argument("--push-scatter", action="store_true",
                    help="push schedule: atomic scatter form of the rounds instead of the gather form")
    ap.add_argument("--no-tail-merge", action="store_true",
                    help="one launch per colour class, never a merged tail")
    ap.add_argument("--persistent", action="store_true",
                    help="SOR as one cooperative launch with grid barriers between colour classes")
    ap.add_argument("--check-every", type=int, default=8,
                    help="sweeps enqueued between host checks of progress")
    ap.add_argument("--skip-below", type=float, default=0.0,
                    help="bound skipping once a sweep updates fewer than this fraction of rows "
                         "(0: the library default, negative: off)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2507_14864_amd as fj

    if args.workload == "batch":
        return bench_batch(args)
    wl = dict(WORKLOADS[args.workload])
    if args.opinions:
        wl["s_kind"] = args.opinions
        wl["desc"] = wl["desc"].split(", s=")[0].split(", s~")[0] + f", s: {args.opinions} (Sec. 6 law)"

    omega_mode = args.omega if args.omega in ("young", "tune") else None
    if args.omega is None:
        omega = wl["omega"] if args.schedule == "sor" else 1.0
    elif omega_mode is None:
        omega = float(args.omega)
    else:
        omega = 1.0  # replaced after ingest
    precision = args.precision or ("fp64" if wl["eps"] < 1e-6 else "fp32")
    dev = "cuda:0"
    t0 = time.perf_counter()
    g, s = make_input(wl)
    log(f"input: n={g.n} nnz={g.nnz} generated in {time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    G = fj.Graph.from_host(g, dev, colour=(args.schedule == "sor"))
    torch.cuda.synchronize()
    ingest_s = time.perf_counter() - t0
    info = G.info()
    log(f"ingest {ingest_s:.2f}s info={info}")
    sd = torch.from_numpy(s).to(dev)
    z = torch.empty(g.n, dtype=torch.float64, device=dev)
    omega_info = None
    if omega_mode == "young":
        t0 = time.perf_counter()
        omega_info = fj.estimate_omega(G, max_iters=5000, tol=1e-6)
        omega = round(omega_info["omega"], 4)
        omega_info["seconds"] = round(time.perf_counter() - t0, 3)
        log(f"omega from mu: {omega_info}")
    elif omega_mode == "tune":
        t0 = time.perf_counter()
        omega_info = fj.tune_omega(G, sd, eps=wl["eps"], precision=precision, schedule=args.schedule,
                                   max_edge_visits=256 * (g.nnz + g.n))
        omega = omega_info["best"]
        omega_info["seconds_total"] = round(time.perf_counter() - t0, 3)
        log(f"omega tuned: {omega_info}")

    def step(profile=False):
        zz, st = fj.solve(G, sd, eps=wl["eps"], omega=omega, precision=precision, schedule=args.schedule,
                          out=z, profile=profile, persistent=args.persistent, gather_bits=args.gather_bits,
                          tail_merge=not args.no_tail_merge,
                          push_scatter="frontier" if args.push_frontier else args.push_scatter,
                          skip_below=args.skip_below, check_every=args.check_every, measures=True)
        return st, st.pop("measures")

    for _ in range(args.warmup):
        st, m = step()
        log(f"warmup: {st}")
    torch.cuda.synchronize()
    times = []
    t_all = time.perf_counter()
    for _ in range(args.steps):
        ta = time.perf_counter()
        st, m = step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ta)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_all
    ms_per_step = 1000.0 * total / max(args.steps, 1)
    log(f"steps: {[round(t * 1000, 2) for t in times]} ms; last stats {st}; metrics {m}")
    # a-posteriori bounds on the measures of the last solve (outside the timed steps)
    mb, bounds, tau = fj.metrics_bounds(G, sd, z, c=1e-5)
    if any(abs(mb[k] - m[k]) > 1e-12 * abs(mb[k]) for k in m):
        raise RuntimeError("measures from the solve differ from fj_metrics_bounds'")
    log(f"metric bounds: tau {tau}; {bounds}")

    roofline = None
    if not args.no_profile:
        # same step with every launch of the iteration kernel bracketed by HIP
        # events on the library's stream
        stp, _ = step(profile=True)
        scatter = args.push_scatter or args.push_frontier
        bytes_total = algorithmic_bytes(args.schedule, stp, g.n, g.nnz, g.w is not None,
                                        gather_rounds=args.schedule == "push" and not scatter,
                                        frontier=args.push_frontier)
        launches = max(stp["kernel_launches"], 1)
        avg_ms = stp["kernel_ms"] / launches
        achieved = bytes_total / (stp["kernel_ms"] * 1e-3) / 1e9
        roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=round(achieved / HBM_PEAK_GBS, 4),
                        traffic=measured_traffic() if args.schedule == "sor" and args.workload == "cl10m" else None,
                        kernel=("k_sor_class" if args.schedule == "sor" or not scatter
                                else "k_frontier_small+k_frontier_big" if args.push_frontier
                                else "k_push_light+k_push_heavy"),
                        algorithmic_bytes_per_launch=int(bytes_total / launches), avg_launch_ms=round(avg_ms, 5),
                        launches=int(stp["kernel_launches"]), kernel_ms=round(stp["kernel_ms"], 3))
        log(f"profiled step: {stp}")
        if args.schedule == "sor":
            # the ceiling of the sweep's memory pattern: the same index stream
            # gathering 4-byte (fixed-point copy) or 8-byte (FP64) values and
            # nothing else; the sweep's arc rate against it
            probe4 = fj.gather_probe(G, 4, 20)
            probe8 = fj.gather_probe(G, 8, 20)
            sweep_rate = stp["edge_visits"] / (stp["kernel_ms"] * 1e-3)
            roofline["gather_ceiling"] = {
                "kernel": "k_gather_probe", "arcs_per_s_4B": round(probe4), "arcs_per_s_8B": round(probe8),
                "sweep_arcs_per_s": round(sweep_rate), "frac": round(sweep_rate / probe4, 4)}
            roofline["gather_frac"] = roofline["gather_ceiling"]["frac"]
            log(f"gather ceiling: {roofline['gather_ceiling']}")

    if args.calib_copy:
        # one elementwise kernel that reads 1 GiB and writes 1 GiB (4x the 256 MB Infinity Cache)
        a = torch.empty(2**30 // 4, dtype=torch.float32, device=dev).fill_(1.0)
        torch.cuda.synchronize()
        b = a + 1.0
        torch.cuda.synchronize()
        log(f"calibration kernel: 1073741824 bytes read, 1073741824 bytes written ({float(b[0])})")

    warm = None
    if not args.no_warm_start and args.workload == "cl10m":
        warm = warm_start_eval(dev)
        log(f"warm start: {warm}")

    batch = None
    if not args.no_batch and args.workload == "cl10m":
        batch = batch_eval(dev, steps=3, warmup=1)
        log(f"batch: {batch}")

    cpu, errors = None, None
    if not args.no_cpu_baseline:
        cpu, zt, z_fifo = cpu_baseline(wl, g, s, st["edge_visits"])
        log(f"cpu baseline: {cpu}")
        errors = {"gpu": errors_vs_exact(g, s, z.cpu().numpy(), zt, wl["eps"]),
                  "oracle_push": errors_vs_exact(g, s, z_fifo, zt, wl["eps"])}
        log(f"errors against the exact z: {errors}")

    value = ms_per_step / 1000.0
    out = {
        "metric": "time to rel. err 1e-4 on 10M-node graph, HBM GB/s; warm vs cold-start speedup",
        "value": round(value, 5),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "n": g.n, "nnz": g.nnz, "eps": wl["eps"], "omega": omega,
                   "omega_choice": omega_mode or "fixed", "omega_search": omega_info,
                   "schedule": args.schedule, "precision": precision, "colours": info["num_colours"],
                   "sweeps_or_rounds": st["rounds"], "merged_tail_classes": st.get("merged_classes", 0),
                   "skipped_row_visits": st.get("skipped_rows", 0), "edge_visits": st["edge_visits"],
                   "bound_atomic_adds": st.get("bound_adds", 0),
                   "certified": st["certified"],
                   "max_ratio": st["max_ratio"], "ingest_s": round(ingest_s, 3),
                   "metrics": {k: m[k] for k in ("P", "D", "I", "C")},
                   "metric_bounds": {"tau": tau, **{k: bounds[k] for k in ("P", "D", "I", "C")}}},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "errors_vs_exact": errors,
        "warm_start": warm,
        "batch": batch,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
