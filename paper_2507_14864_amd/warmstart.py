"""Training and evaluation of the learned warm start (an extension; the
paper's method is the push that runs after it).

Training set: 64 directed Chung-Lu graphs (out/in exponent 2.1, 10 arc
samples per node, weights U[0.5, 1.5]) with node counts log-uniform in
[100k, 1M] (seeds 1000-1063); opinions cycle through U[0,1], Beta(2,2) and
the bimodal 0.5 Beta(2,8) + 0.5 Beta(8,2); targets are FP64 solves of the same
problem to eps = 1e-6.  The stored weights come from 150 epochs with the
relative loss weights 1 / (z + 3e-3)^2, chosen among 60-300 epochs and floors
1e-3 to 1e-2 by the time to the certificate on a validation graph (2M nodes,
20M arc samples, seed 7777).  Held out: a directed Chung-Lu graph with 5M
nodes and 50M arc samples (seed 9999) with bimodal opinions.

All arithmetic runs in libfj's kernels (forward, backward, Adam, solves);
this module only sequences the calls and times them.
"""
import os
import time

import numpy as np
import torch

from . import fj

PARAMS_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "wsnet_params.npy")
TRAIN_SEEDS = range(1000, 1064)
HELDOUT_SEED = 9999
S_KINDS = ("uniform", "beta", "bimodal")


def _synth():
    import synth
    return synth


def training_problem(i: int):
    """The i-th training graph (host CSR) and its opinions."""
    synth = _synth()
    seed = TRAIN_SEEDS[i]
    rng = np.random.default_rng(seed)
    n = int(round(np.exp(rng.uniform(np.log(100_000), np.log(1_000_000)))))
    g = synth.chung_lu(n, 10 * n, 2.1, seed, directed=True, weighted=True)
    kind = S_KINDS[i % 3]
    s = synth.opinions(n, kind, seed, a=2, b=2) if kind == "beta" else synth.opinions(n, kind, seed)
    return g, s


VALIDATION_SEED = 7777


def validation_problem(n: int = 2_000_000, m: int = 20_000_000):
    """A directed graph of the training law, 2M nodes, bimodal opinions: used
    to choose the training settings, so the held-out graph only reports."""
    synth = _synth()
    g = synth.chung_lu(n, m, 2.1, VALIDATION_SEED, directed=True, weighted=True)
    return g, synth.opinions(n, "bimodal", VALIDATION_SEED)


def heldout_problem(n: int = 5_000_000, m: int = 50_000_000):
    synth = _synth()
    g = synth.chung_lu(n, m, 2.1, HELDOUT_SEED, directed=True, weighted=True)
    return g, synth.opinions(n, "bimodal", HELDOUT_SEED)


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights, zero biases, in the flat layout of fj_wsnet_*:
    W1 (8x64), b1 (64), Wp (64x16), W2 (80x64), b2 (64), u (64), c0 (1)."""
    rng = np.random.default_rng(seed)
    w1 = rng.normal(0, np.sqrt(2.0 / 8), 8 * 64)
    wp = rng.normal(0, np.sqrt(1.0 / 64), 64 * 16)
    w2 = rng.normal(0, np.sqrt(2.0 / 80), 80 * 64)
    u = rng.normal(0, np.sqrt(1.0 / 64), 64)
    return np.concatenate([w1, np.zeros(64), wp, w2, np.zeros(64), u, np.zeros(1)]).astype(np.float32)


def train(num_graphs: int = 64, epochs: int = 150, lr: float = 3e-3, device: str = "cuda:0", log=print,
          seed: int = 0, decay: float = 0.95, rel_floor: float = 3e-3):
    """Train on solver-generated targets, the step size times `decay` after
    every epoch; rel_floor > 0 weighs each node's squared error by
    1 / (z + rel_floor)^2.  Returns (params, loss history)."""
    data = []
    t0 = time.perf_counter()
    for i in range(num_graphs):
        g, s = training_problem(i)
        G = fj.Graph.from_host(g, device)
        sd = torch.from_numpy(s).to(device)
        zt, st = fj.solve(G, sd, eps=1e-6, omega=1.0, schedule="push", precision="fp64")
        data.append((G, sd, zt.clone()))
    log(f"warm start: {num_graphs} training targets solved in {time.perf_counter() - t0:.1f}s")
    params = torch.from_numpy(init_params(seed)).to(device)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    rng = np.random.default_rng(seed)
    hist, step = [], 0
    t0 = time.perf_counter()
    for ep in range(epochs):
        rate = lr * (decay ** ep)
        for i in rng.permutation(len(data)):
            G, sd, zt = data[i]
            step += 1
            loss = fj.wsnet_train_step(G, sd, zt, params, m, v, step, rate, rel_floor)
            hist.append(loss)
        ep_loss = float(torch.stack(hist[-len(data):]).mean().item())
        log(f"warm start: epoch {ep} mean loss {ep_loss:.3e}")
    torch.cuda.synchronize()
    log(f"warm start: {step} Adam steps in {time.perf_counter() - t0:.1f}s")
    return params, [float(x.item()) for x in hist]


def save_params(params: torch.Tensor, path: str = PARAMS_PATH):
    np.save(path, params.detach().cpu().numpy().astype(np.float32), allow_pickle=False)


def load_params(device: str = "cuda:0", path: str = PARAMS_PATH):
    if not os.path.exists(path):
        return None
    return torch.from_numpy(np.load(path, allow_pickle=False).astype(np.float32)).to(device)


def _timed(fn, reps: int = 3):
    out, best = None, None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    return out, best


def evaluate(G, sd: torch.Tensor, params, eps: float = 1e-4, omega: float = 1.0, reps: int = 3,
             jacobi=(2, 4, 8)):
    """Time to the same certificate from a cold start, from the network's
    proposal (inference included), and from the untrained controls z0 = s and
    z0 = k synchronous FJ steps (Eq. (1)) from s (their steps included)."""
    res = {}

    def cold():
        return fj.solve(G, sd, eps=eps, omega=omega, schedule="sor")

    (z_c, st_c), t_cold = _timed(cold, reps)
    res["cold"] = dict(s=t_cold, sweeps=st_c["rounds"], certified=st_c["certified"])
    z0buf = torch.empty_like(sd)

    def warm():
        z0 = fj.wsnet_forward(G, sd, params, out=z0buf)
        return fj.solve(G, sd, eps=eps, omega=omega, schedule="sor", z0=z0)

    if params is not None:
        (z_w, st_w), t_warm = _timed(warm, reps)
        _, t_inf = _timed(lambda: fj.wsnet_forward(G, sd, params, out=z0buf), reps)
        zc = z_c.cpu().numpy()
        z0 = z0buf.cpu().numpy()
        res["net"] = dict(s=t_warm, inference_s=t_inf, sweeps=st_w["rounds"], certified=st_w["certified"],
                          z0_rel_err_median=float(np.median(np.abs(z0 - zc) / np.abs(zc).clip(1e-5))),
                          z0_rel_err_max=float(np.max(np.abs(z0 - zc) / np.abs(zc).clip(1e-5))))

    def from_s():
        return fj.solve(G, sd, eps=eps, omega=omega, schedule="sor", z0=sd)

    (_, st_s), t_s = _timed(from_s, reps)
    res["z0=s"] = dict(s=t_s, sweeps=st_s["rounds"], certified=st_s["certified"])
    for k in jacobi:
        def jac():
            z0 = sd.clone()
            fj.jacobi_steps(G, sd, z0, k)
            return fj.solve(G, sd, eps=eps, omega=omega, schedule="sor", z0=z0)
        (_, st_j), t_j = _timed(jac, reps)
        res[f"z0=jacobi{k}"] = dict(s=t_j, sweeps=st_j["rounds"], certified=st_j["certified"])
    if "net" in res:
        res["speedup_net_vs_cold"] = t_cold / res["net"]["s"]
        best_ctrl = min(v["s"] for k, v in res.items() if k.startswith("z0="))
        res["speedup_net_vs_best_control"] = best_ctrl / res["net"]["s"]
    return res


def main():
    """Train, store the weights beside this module, and evaluate on the held-out graph."""
    import json
    import sys
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    params, hist = train(log=log)
    save_params(params)
    g, s = heldout_problem()
    G = fj.Graph.from_host(g, "cuda:0", colour=True)
    sd = torch.from_numpy(s).to("cuda:0")
    for omega in (1.0, 1.1, 1.2):
        res = evaluate(G, sd, params, omega=omega)
        print(json.dumps({"omega": omega, **res}), flush=True)


if __name__ == "__main__":
    main()
