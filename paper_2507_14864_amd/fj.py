"""Python binding of libfj.so (include/fj.h): argument marshalling only.

Every step of the solve runs in the library's HIP kernels.  PyTorch supplies
device memory (workspaces are torch uint8 tensors) and the current stream.
There is no CPU fallback: without the built library or a GPU every call raises.
"""
import ctypes
import sys
import os
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfj.so")

FJ_OK, FJ_ERR_INVALID_ARGUMENT, FJ_ERR_WORKSPACE_TOO_SMALL = 0, 1, 2
FJ_ERR_NOT_CONVERGED, FJ_ERR_HIP, FJ_ERR_UNSUPPORTED = 3, 4, 5
FJ_GRAPH_COLOUR = 1
FJ_FP32, FJ_FP64 = 0, 1
SCHEDULES = {"auto": 0, "push": 1, "sor": 2}
PRECISIONS = {"fp32": FJ_FP32, "fp64": FJ_FP64}


class FJError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"[fj status {status}] {message}")
        self.status = status


class FJNotConverged(FJError):
    """The work cap or refinement budget ran out; ``z`` and ``stats`` hold the
    last estimate."""

    def __init__(self, status, message, z=None, stats=None):
        super().__init__(status, message)
        self.z = z
        self.stats = stats


class GraphDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("w", ctypes.c_void_p), ("directed", ctypes.c_int32)]


class GraphInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("directed", ctypes.c_int32),
                ("weighted", ctypes.c_int32), ("max_degree", ctypes.c_int32),
                ("max_in_degree", ctypes.c_int32), ("num_colours", ctypes.c_int32),
                ("colour_rounds", ctypes.c_int32)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("omega", ctypes.c_double), ("c", ctypes.c_double),
                ("sigma", ctypes.c_double), ("precision", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("max_edge_visits", ctypes.c_int64), ("max_refinements", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("z0", ctypes.c_void_p), ("profile", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("gather_bits", ctypes.c_int32), ("push_scatter", ctypes.c_int32),
                ("no_tail_merge", ctypes.c_int32), ("skip_below", ctypes.c_double), ("measures", ctypes.c_void_p)]


class SolveStats(ctypes.Structure):
    _fields_ = [("pushes", ctypes.c_int64), ("edge_visits", ctypes.c_int64), ("rounds", ctypes.c_int64),
                ("launches", ctypes.c_int64), ("refinements", ctypes.c_int32), ("certified", ctypes.c_int32),
                ("max_ratio", ctypes.c_double), ("seconds", ctypes.c_double), ("kernel_ms", ctypes.c_double),
                ("kernel_launches", ctypes.c_int64), ("num_colours", ctypes.c_int32),
                ("mirror_rounds", ctypes.c_int64), ("merged_classes", ctypes.c_int32),
                ("skipped_rows", ctypes.c_int64), ("skipped_arcs", ctypes.c_int64),
                ("mirror_edge_visits", ctypes.c_int64), ("bound_adds", ctypes.c_int64),
                ("mirror_fp64_edge_visits", ctypes.c_int64)]

    def to_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class MetricsOut(ctypes.Structure):
    _fields_ = [("P", ctypes.c_double), ("D", ctypes.c_double), ("I", ctypes.c_double),
                ("C", ctypes.c_double), ("mean", ctypes.c_double)]


_LIB = None


def lib():
    """Load libfj.so (raises if it was not built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, sz, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_double
        P = ctypes.POINTER
        L.fj_last_error.restype = ctypes.c_char_p
        L.fj_version.restype = i32
        L.fj_graph_workspace_bytes.argtypes = [P(GraphDesc), i32]
        L.fj_graph_workspace_bytes.restype = sz
        L.fj_graph_create.argtypes = [P(GraphDesc), i32, vp, sz, vp, P(vp)]
        L.fj_graph_create.restype = i32
        L.fj_graph_destroy.argtypes = [vp]
        L.fj_graph_destroy.restype = i32
        L.fj_graph_get_info.argtypes = [vp, P(GraphInfo)]
        L.fj_graph_get_info.restype = i32
        L.fj_graph_colour_sizes.argtypes = [vp, vp]
        L.fj_graph_colour_sizes.restype = i32
        L.fj_graph_colours.argtypes = [vp, vp, vp]
        L.fj_graph_colours.restype = i32
        L.fj_solve_workspace_bytes.argtypes = [vp, P(SolveOpts)]
        L.fj_solve_workspace_bytes.restype = sz
        L.fj_solve.argtypes = [vp, vp, P(SolveOpts), vp, vp, sz, P(SolveStats), vp]
        L.fj_solve.restype = i32
        L.fj_metrics_workspace_bytes.argtypes = [vp]
        L.fj_metrics_workspace_bytes.restype = sz
        L.fj_metrics.argtypes = [vp, vp, vp, P(MetricsOut), vp, sz, vp]
        L.fj_metrics.restype = i32
        L.fj_metrics_noalloc_max_bytes.argtypes = []
        L.fj_metrics_noalloc_max_bytes.restype = sz
        L.fj_metrics_noalloc_bytes.argtypes = [vp]
        L.fj_metrics_noalloc_bytes.restype = sz
        L.fj_metrics_noalloc.argtypes = [vp, vp, vp, P(MetricsOut), vp]
        L.fj_metrics_noalloc.restype = i32
        L.fj_gather_probe_workspace_bytes.argtypes = [vp]
        L.fj_gather_probe_workspace_bytes.restype = sz
        L.fj_gather_probe.argtypes = [vp, i32, i32, P(dbl), vp, sz, vp]
        L.fj_gather_probe.restype = i32
        L.fj_metrics_bounds.argtypes = [vp, vp, vp, ctypes.c_double, P(MetricsOut), P(MetricsOut),
                                        P(ctypes.c_double), vp, sz, vp]
        L.fj_metrics_bounds.restype = i32
        L.fj_optimal_omega.argtypes = [dbl]
        L.fj_optimal_omega.restype = dbl
        L.fj_omega_workspace_bytes.argtypes = [vp]
        L.fj_omega_workspace_bytes.restype = sz
        L.fj_estimate_omega.argtypes = [vp, i32, dbl, P(dbl), P(dbl), P(i32), vp, sz, vp]
        L.fj_estimate_omega.restype = i32
        L.fj_tune_omega.argtypes = [vp, vp, P(SolveOpts), P(dbl), i32, P(ctypes.c_int64), P(dbl), P(dbl), vp,
                                    vp, sz, vp]
        L.fj_tune_omega.restype = i32
        L.fj_stress_workspace_bytes.argtypes = [vp]
        L.fj_stress_workspace_bytes.restype = sz
        L.fj_stress.argtypes = [vp, vp, vp, vp, P(dbl), vp, sz, vp]
        L.fj_stress.restype = i32
        L.fj_certify.argtypes = [vp, vp, vp, dbl, dbl, dbl, P(dbl), vp, sz, vp]
        L.fj_certify.restype = i32
        _LIB = L
    return _LIB


def _check(rc: int):
    if rc != FJ_OK:
        msg = lib().fj_last_error().decode(errors="replace")
        raise FJError(rc, msg)


def _stream() -> ctypes.c_void_p:
    if not torch.cuda.is_available():
        raise RuntimeError("libfj needs a ROCm GPU; none is visible")
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_ptr(t: Optional[torch.Tensor], dtype, n: int, name: str):
    if t is None:
        return None
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name}: need a contiguous {dtype} CUDA tensor of {n} elements")
    return ctypes.c_void_p(t.data_ptr())


def _workspace(nbytes: int, device) -> torch.Tensor:
    # torch's caching allocator returns blocks aligned to at least 512 bytes
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


class Graph:
    """A graph resident on the GPU plus the library's ingest products.

    ``row_ptr``/``col``/``w`` are CUDA tensors (int32, int32, float32 or None)
    holding CSR(A): row i lists j with a_ij > 0.  They are kept alive here.
    """

    def __init__(self, row_ptr: torch.Tensor, col: torch.Tensor, w: Optional[torch.Tensor] = None,
                 directed: bool = False, colour: bool = False):
        n = row_ptr.numel() - 1
        nnz = col.numel()
        self.n, self.nnz, self.directed = n, nnz, bool(directed)
        self.row_ptr, self.col, self.w = row_ptr, col, w
        self.device = row_ptr.device
        desc = GraphDesc(n, nnz, _dev_ptr(row_ptr, torch.int32, n + 1, "row_ptr"),
                         _dev_ptr(col, torch.int32, nnz, "col"),
                         _dev_ptr(w, torch.float32, nnz, "w") if w is not None else None,
                         1 if directed else 0)
        flags = FJ_GRAPH_COLOUR if colour else 0
        L = lib()
        nbytes = L.fj_graph_workspace_bytes(ctypes.byref(desc), flags)
        self.ws = _workspace(nbytes, self.device)
        h = ctypes.c_void_p()
        self._h = None
        _check(L.fj_graph_create(ctypes.byref(desc), flags, ctypes.c_void_p(self.ws.data_ptr()),
                                 self.ws.numel(), _stream(), ctypes.byref(h)))
        self._h = h
        self._solve_ws = None
        self._metrics_ws = None

    @classmethod
    def from_host(cls, g, device="cuda", colour: bool = False) -> "Graph":
        """From a host CSR (``synth.CSRGraph`` or anything with n, row_ptr,
        col, w, directed)."""
        rp = torch.from_numpy(g.row_ptr).to(device)
        col = torch.from_numpy(g.col).to(device)
        w = None if g.w is None else torch.from_numpy(g.w).to(device)
        return cls(rp, col, w, directed=g.directed, colour=colour)

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        out = GraphInfo()
        _check(lib().fj_graph_get_info(self._h, ctypes.byref(out)))
        return {k: getattr(out, k) for k, _ in out._fields_}

    def colour_sizes(self):
        k = self.info()["num_colours"]
        buf = (ctypes.c_int64 * max(k, 1))()
        _check(lib().fj_graph_colour_sizes(self._h, buf))
        return [int(buf[i]) for i in range(k)]

    def colours(self) -> torch.Tensor:
        out = torch.empty(self.n, dtype=torch.int32, device=self.device)
        _check(lib().fj_graph_colours(self._h, ctypes.c_void_p(out.data_ptr()), _stream()))
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _LIB is not None:
            _LIB.fj_graph_destroy(h)
            self._h = None


def _scatter_mode(push_scatter) -> int:
    """push_scatter: False/0 gather-form rounds, True/1 atomic scatter over a
    scan of all nodes, "frontier"/2 atomic scatter over a frontier queue."""
    if push_scatter == "frontier":
        return 2
    if isinstance(push_scatter, bool):
        return 1 if push_scatter else 0
    return int(push_scatter)


def make_opts(eps=1e-4, omega=1.0, c=1e-5, sigma=1e-5, precision="fp32", schedule="auto",
              max_edge_visits=0, max_refinements=-1, check_every=8, z0=None, profile=False,
              persistent=False, gather_bits=0, tail_merge=True, push_scatter=False,
              skip_below=0.0) -> SolveOpts:
    return SolveOpts(float(eps), float(omega), float(c), float(sigma), PRECISIONS[precision],
                     SCHEDULES[schedule], int(max_edge_visits), int(max_refinements), int(check_every),
                     None if z0 is None else ctypes.c_void_p(z0.data_ptr()), 1 if profile else 0,
                     1 if persistent else 0, int(gather_bits), _scatter_mode(push_scatter), 0 if tail_merge else 1,
                     float(skip_below))


def solve(graph: Graph, s: torch.Tensor, eps: float = 1e-4, omega: float = 1.0, c: float = 1e-5,
          sigma: float = 1e-5, precision: str = "fp32", schedule: str = "auto", max_edge_visits: int = 0,
          max_refinements: int = -1, check_every: int = 8, z0: Optional[torch.Tensor] = None,
          out: Optional[torch.Tensor] = None, profile: bool = False, persistent: bool = False,
          gather_bits: int = 0, tail_merge: bool = True, push_scatter: bool = False,
          skip_below: float = 0.0, measures: bool = False):
    """ImprovedBLISOR on the GPU.  Returns (z, stats dict).

    measures: also the Table 1 measures of z in stats["measures"]
    (fj_solve_opts.measures; the SOR schedule forms D in its final
    certificate's gather pass).  Raises FJNotConverged (with .z and .stats)
    when the certificate could not be reached."""
    n = graph.n
    _dev_ptr(s, torch.float64, n, "s")
    if z0 is not None:
        _dev_ptr(z0, torch.float64, n, "z0")
    z = out if out is not None else torch.empty(n, dtype=torch.float64, device=graph.device)
    _dev_ptr(z, torch.float64, n, "out")
    opts = make_opts(eps, omega, c, sigma, precision, schedule, max_edge_visits, max_refinements,
                     check_every, z0, profile, persistent, gather_bits, tail_merge, push_scatter, skip_below)
    mo = MetricsOut() if measures else None
    if mo is not None:
        opts.measures = ctypes.addressof(mo)
    L = lib()
    nbytes = L.fj_solve_workspace_bytes(graph.handle, ctypes.byref(opts))
    if graph._solve_ws is None or graph._solve_ws.numel() < nbytes:
        graph._solve_ws = _workspace(nbytes, graph.device)
    ws = graph._solve_ws
    st = SolveStats()
    rc = L.fj_solve(graph.handle, ctypes.c_void_p(s.data_ptr()), ctypes.byref(opts),
                    ctypes.c_void_p(z.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                    ctypes.byref(st), _stream())
    stats = st.to_dict()
    if mo is not None and rc in (FJ_OK, FJ_ERR_NOT_CONVERGED):
        stats["measures"] = {k: getattr(mo, k) for k, _ in mo._fields_}
    if rc == FJ_ERR_NOT_CONVERGED:
        raise FJNotConverged(rc, L.fj_last_error().decode(errors="replace"), z, stats)
    _check(rc)
    return z, stats


def _metrics_ws(graph: Graph) -> torch.Tensor:
    nbytes = lib().fj_metrics_workspace_bytes(graph.handle)
    if graph._metrics_ws is None or graph._metrics_ws.numel() < nbytes:
        graph._metrics_ws = _workspace(nbytes, graph.device)
    return graph._metrics_ws


def metrics(graph: Graph, s: torch.Tensor, z: torch.Tensor) -> dict:
    """Table 1 measures P, D, I, C (and the mean of z), FP64, reproducible."""
    n = graph.n
    _dev_ptr(s, torch.float64, n, "s")
    _dev_ptr(z, torch.float64, n, "z")
    ws = _metrics_ws(graph)
    out = MetricsOut()
    _check(lib().fj_metrics(graph.handle, ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(z.data_ptr()),
                            ctypes.byref(out), ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return {k: getattr(out, k) for k, _ in out._fields_}


def metrics_noalloc(graph: Graph, s: torch.Tensor, z: torch.Tensor) -> dict:
    """fj_metrics_noalloc: the measures with the partial sums in the library's
    static device array (no workspace; graphs up to its size)."""
    n = graph.n
    _dev_ptr(s, torch.float64, n, "s")
    _dev_ptr(z, torch.float64, n, "z")
    out = MetricsOut()
    _check(lib().fj_metrics_noalloc(graph.handle, ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(z.data_ptr()),
                                    ctypes.byref(out), _stream()))
    return {k: getattr(out, k) for k, _ in out._fields_}


def metrics_noalloc_bytes(graph: Graph) -> tuple:
    """(bytes of the static array this graph needs, the array's size)."""
    return int(lib().fj_metrics_noalloc_bytes(graph.handle)), int(lib().fj_metrics_noalloc_max_bytes())


def metrics_bounds(graph: Graph, s: torch.Tensor, z: torch.Tensor, c: float = 1e-5) -> tuple:
    """The measures of z, a-posteriori bounds on their distance from those of
    the exact solution (from the residual level tau by Lemma 7), and tau."""
    n = graph.n
    _dev_ptr(s, torch.float64, n, "s")
    _dev_ptr(z, torch.float64, n, "z")
    ws = _metrics_ws(graph)
    out, bound, tau = MetricsOut(), MetricsOut(), ctypes.c_double()
    _check(lib().fj_metrics_bounds(graph.handle, ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(z.data_ptr()),
                                   float(c), ctypes.byref(out), ctypes.byref(bound), ctypes.byref(tau),
                                   ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return ({k: getattr(out, k) for k, _ in out._fields_}, {k: getattr(bound, k) for k, _ in bound._fields_},
            tau.value)


def gather_probe(graph: Graph, value_bytes: int = 4, reps: int = 10) -> float:
    """Arcs per second of the sweep's gather pattern alone (fj_gather_probe)."""
    ws = _workspace(lib().fj_gather_probe_workspace_bytes(graph.handle), graph.device)
    rate = ctypes.c_double()
    _check(lib().fj_gather_probe(graph.handle, int(value_bytes), int(reps), ctypes.byref(rate),
                                 ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return rate.value


def optimal_omega(mu: float) -> float:
    """Eq. (optimal-omega) for a given spectral radius mu."""
    return lib().fj_optimal_omega(float(mu))


def estimate_omega(graph: Graph, max_iters: int = 2000, tol: float = 1e-7) -> dict:
    """mu = rho((I+D)^{-1} A) by power iteration on the GPU and the omega of
    Eq. (optimal-omega) for it."""
    ws = _workspace(lib().fj_omega_workspace_bytes(graph.handle), graph.device)
    mu, om, it = ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
    _check(lib().fj_estimate_omega(graph.handle, int(max_iters), float(tol), ctypes.byref(mu), ctypes.byref(om),
                                   ctypes.byref(it), ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return {"mu": mu.value, "omega": om.value, "iters": it.value}


def tune_omega(graph: Graph, s: torch.Tensor, omegas=None, **opts) -> dict:
    """The paper's heuristic: solve once per candidate omega (default 1.95
    down to 1.0 in steps of 0.05) and keep the one with the fewest updates."""
    if omegas is None:
        omegas = [round(1.95 - 0.05 * k, 2) for k in range(20)]
    n = graph.n
    _dev_ptr(s, torch.float64, n, "s")
    o = make_opts(**opts)
    ws = _workspace(lib().fj_solve_workspace_bytes(graph.handle, ctypes.byref(o)), graph.device)
    z = torch.empty(n, dtype=torch.float64, device=graph.device)
    k = len(omegas)
    om = (ctypes.c_double * k)(*omegas)
    upd = (ctypes.c_int64 * k)()
    secs = (ctypes.c_double * k)()
    best = ctypes.c_double()
    _check(lib().fj_tune_omega(graph.handle, ctypes.c_void_p(s.data_ptr()), ctypes.byref(o), om, k, upd, secs,
                               ctypes.byref(best), ctypes.c_void_p(z.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                               ws.numel(), _stream()))
    return {"best": best.value, "omegas": list(omegas), "updates": list(upd), "seconds": list(secs)}


def stress(graph: Graph, s: torch.Tensor, z: torch.Tensor, per_node: bool = True):
    """Stress of every node, (z_i - s_i)^2 + sum_j a_ij (z_i - z_j)^2, and
    their total (FP64, reproducible).  Returns (vector or None, total)."""
    n = graph.n
    _dev_ptr(s, torch.float64, n, "s")
    _dev_ptr(z, torch.float64, n, "z")
    nbytes = lib().fj_stress_workspace_bytes(graph.handle)
    ws = _workspace(nbytes, graph.device)
    vec = torch.empty(n, dtype=torch.float64, device=graph.device) if per_node else None
    total = ctypes.c_double()
    _check(lib().fj_stress(graph.handle, ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(z.data_ptr()),
                           ctypes.c_void_p(vec.data_ptr() if vec is not None else None), ctypes.byref(total),
                           ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return vec, total.value


def certify(graph: Graph, s: torch.Tensor, z: torch.Tensor, eps: float, c: float = 1e-5,
            sigma: float = 1e-5) -> float:
    """max_v |s_v - ((I+L) z)_v| / (eps' (s_v + c)) in FP64 on the GPU."""
    n = graph.n
    _dev_ptr(s, torch.float64, n, "s")
    _dev_ptr(z, torch.float64, n, "z")
    ws = _metrics_ws(graph)
    out = ctypes.c_double()
    _check(lib().fj_certify(graph.handle, ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(z.data_ptr()),
                            float(eps), float(c), float(sigma), ctypes.byref(out),
                            ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return out.value


# ---------------------------------------------------------------- batched solve
class BatchItemDesc(ctypes.Structure):
    _fields_ = [("graph", GraphDesc), ("k", ctypes.c_int32)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("omega", ctypes.c_double), ("omega_undirected", ctypes.c_double),
                ("omega_directed", ctypes.c_double), ("omega_multi", ctypes.c_double),
                ("sweep_budget", ctypes.c_int32), ("graph_nodes", ctypes.c_int32),
                ("num_colours", ctypes.c_int32), ("tune_ms", ctypes.c_double * 16),
                ("union_chunks_in_flight", ctypes.c_int32), ("multi_arcs_in_flight", ctypes.c_int32),
                ("cache_hit", ctypes.c_int32), ("bound", ctypes.c_int32)]


def batch_tune_cache_clear():
    """Forget the batch shapes fj_batch_tune has kept in this process."""
    _batch_lib().fj_batch_tune_cache_clear()


def _batch_lib():
    L = lib()
    if not getattr(L, "_batch_ready", False):
        vp, i32, sz, P = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t, ctypes.POINTER
        L.fj_batch_workspace_bytes.argtypes = [P(BatchItemDesc), i32]
        L.fj_batch_workspace_bytes.restype = sz
        L.fj_batch_create.argtypes = [P(BatchItemDesc), i32, P(SolveOpts), vp, sz, vp, P(vp)]
        L.fj_batch_create.restype = i32
        L.fj_batch_destroy.argtypes = [vp]
        L.fj_batch_destroy.restype = i32
        L.fj_batch_io.argtypes = [vp, i32, P(ctypes.c_void_p), P(ctypes.c_void_p)]
        L.fj_batch_io.restype = i32
        L.fj_batch_tune.argtypes = [vp, P(ctypes.c_double), i32, vp]
        L.fj_batch_tune.restype = i32
        L.fj_batch_get_info.argtypes = [vp, P(BatchInfo)]
        L.fj_batch_get_info.restype = i32
        L.fj_batch_set_omegas.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.fj_batch_set_omegas.restype = i32
        L.fj_batch_set_launch.argtypes = [vp, i32, i32]
        L.fj_batch_set_launch.restype = i32
        L.fj_solve_batched.argtypes = [vp, vp, vp, vp]
        L.fj_solve_batched.restype = i32
        L.fj_batch_tune_cache_clear.argtypes = []
        L.fj_batch_tune_cache_clear.restype = None
        L.fj_batch_bind.argtypes = [vp, vp, vp, vp]
        L.fj_batch_bind.restype = i32
        L.fj_batch_check.argtypes = [vp, i32, P(i32), vp, vp, vp]
        L.fj_batch_check.restype = i32
        L._batch_ready = True
    return L


class Batch:
    """Many graphs and opinion vectors solved by one enqueued sequence
    (fj_solve_batched).  ``graphs`` is a list of (row_ptr, col, w, directed)
    with CUDA tensors; ``ks`` the number of vectors per graph (1..64)."""

    def __init__(self, graphs, ks, eps=1e-4, omega=1.5, c=1e-5, sigma=1e-5):
        L = _batch_lib()
        self._keep = []
        self._bound = None
        self.ns, self.ks = [], [int(k) for k in ks]
        descs = (BatchItemDesc * len(graphs))()
        for i, (rp, col, w, directed) in enumerate(graphs):
            n = rp.numel() - 1
            self.ns.append(n)
            self._keep += [rp, col, w]
            descs[i].graph = GraphDesc(n, col.numel(), _dev_ptr(rp, torch.int32, n + 1, "row_ptr"),
                                       _dev_ptr(col, torch.int32, col.numel(), "col"),
                                       _dev_ptr(w, torch.float32, col.numel(), "w") if w is not None else None,
                                       1 if directed else 0)
            descs[i].k = self.ks[i]
        self._descs = descs
        self.device = graphs[0][0].device
        nbytes = L.fj_batch_workspace_bytes(descs, len(graphs))
        if nbytes == 0:
            raise ValueError("invalid batch description")
        self.ws = _workspace(nbytes, self.device)
        opts = make_opts(eps=eps, omega=omega, c=c, sigma=sigma)
        h = ctypes.c_void_p()
        self._h = None
        _check(L.fj_batch_create(descs, len(graphs), ctypes.byref(opts), ctypes.c_void_p(self.ws.data_ptr()),
                                 self.ws.numel(), _stream(), ctypes.byref(h)))
        self._h = h
        self.num_items = len(graphs)
        self._stats = torch.empty(self.num_items * ctypes.sizeof(SolveStats), dtype=torch.uint8, device=self.device)
        self._mets = torch.empty(sum(self.ks) * ctypes.sizeof(MetricsOut), dtype=torch.uint8, device=self.device)

    def _view(self, ptr, i):
        off = ptr - self.ws.data_ptr()
        n, k = self.ns[i], self.ks[i]
        t = self.ws[off:off + 8 * n * k].view(torch.float64)
        return t.view(n, k) if k > 1 else t

    def input(self, i) -> torch.Tensor:
        """Writable view of item i's opinions ([n] or [n][k] node-major)."""
        s, z = ctypes.c_void_p(), ctypes.c_void_p()
        _check(_batch_lib().fj_batch_io(self._h, i, ctypes.byref(s), ctypes.byref(z)))
        return self._view(s.value, i)

    def output(self, i) -> torch.Tensor:
        s, z = ctypes.c_void_p(), ctypes.c_void_p()
        _check(_batch_lib().fj_batch_io(self._h, i, ctypes.byref(s), ctypes.byref(z)))
        return self._view(z.value, i)

    def tune(self, omegas=(1.0, 1.2, 1.4, 1.5, 1.6, 1.7)):
        arr = (ctypes.c_double * len(omegas))(*omegas)
        _check(_batch_lib().fj_batch_tune(self._h, arr, len(omegas), _stream()))
        return self.info()

    def set_launch(self, union_chunks=0, multi_arcs=0):
        """Override the tuned launch parameters (union_chunks 2, 4 or 8;
        multi_arcs 4, 8 or 16; 0 keeps); a recorded graph is recorded again.
        Results are unchanged bit for bit."""
        _check(_batch_lib().fj_batch_set_launch(self._h, int(union_chunks), int(multi_arcs)))

    def set_omegas(self, undirected=0.0, directed=0.0, multi=0.0):
        """Per-group relaxation factors (<= 0 keeps a group's value); drops
        the recorded graph."""
        _check(_batch_lib().fj_batch_set_omegas(self._h, float(undirected), float(directed), float(multi)))

    def info(self) -> dict:
        out = BatchInfo()
        _check(_batch_lib().fj_batch_get_info(self._h, ctypes.byref(out)))
        d = {k: getattr(out, k) for k, _ in out._fields_ if k != "tune_ms"}
        d["tune_ms"] = list(out.tune_ms)
        return d

    def solve_async(self):
        """Enqueue one batched solve on the current stream (no host sync)."""
        _check(_batch_lib().fj_solve_batched(self._h, ctypes.c_void_p(self._stats.data_ptr()),
                                             ctypes.c_void_p(self._mets.data_ptr()), _stream()))

    def results(self):
        """(stats per item, measures per item and vector) after a solve."""
        import numpy as np
        torch.cuda.current_stream().synchronize()
        st_raw = self._stats.cpu().numpy().tobytes()
        me_raw = self._mets.cpu().numpy().tobytes()
        stats = [SolveStats.from_buffer_copy(st_raw, i * ctypes.sizeof(SolveStats)).to_dict()
                 for i in range(self.num_items)]
        mets, off = [], 0
        for i, k in enumerate(self.ks):
            row = []
            for q in range(k):
                m = MetricsOut.from_buffer_copy(me_raw, (off + q) * ctypes.sizeof(MetricsOut))
                row.append({f: getattr(m, f) for f, _ in m._fields_})
            mets.append(row)
            off += k
        return stats, mets

    def solve(self):
        self.solve_async()
        return self.results()

    def bind(self, s_list=None, z_list=None):
        """Caller-owned inputs and outputs (fj_batch_bind): item i reads
        s_list[i] and writes z_list[i] (contiguous float64 CUDA tensors of
        n_i * k_i elements, node-major).  No arguments: unbind."""
        if s_list is None:
            self._bound = None
            _check(_batch_lib().fj_batch_bind(self._h, None, None, _stream()))
            return
        if len(s_list) != self.num_items or len(z_list) != self.num_items:
            raise ValueError("need one s and one z tensor per item")
        for i, (si, zi) in enumerate(zip(s_list, z_list)):
            cnt = self.ns[i] * self.ks[i]
            for t, nm in ((si, "s"), (zi, "z")):
                if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous() or t.numel() != cnt:
                    raise ValueError(f"item {i}: {nm} must be a contiguous float64 CUDA tensor of {cnt} elements")
        sp = (ctypes.c_void_p * self.num_items)(*[t.data_ptr() for t in s_list])
        zp = (ctypes.c_void_p * self.num_items)(*[t.data_ptr() for t in z_list])
        self._bound = (list(s_list), list(z_list))  # keep the buffers alive while bound
        _check(_batch_lib().fj_batch_bind(self._h, sp, zp, _stream()))

    def check(self, extra_sweeps: int = 256) -> int:
        """fj_batch_check after a solve: items whose certificate failed sweep
        on for up to extra_sweeps more sweeps; refreshes results().  Returns
        the number of items still not certified (0 on success)."""
        cnt = ctypes.c_int32()
        rc = _batch_lib().fj_batch_check(self._h, int(extra_sweeps), ctypes.byref(cnt),
                                         ctypes.c_void_p(self._stats.data_ptr()),
                                         ctypes.c_void_p(self._mets.data_ptr()), _stream())
        if rc not in (FJ_OK, FJ_ERR_NOT_CONVERGED):
            _check(rc)
        return int(cnt.value)

    def close(self):
        """Release the batch (its recorded hipGraph included) now."""
        h = getattr(self, "_h", None)
        if h is not None and _LIB is not None:
            _LIB.fj_batch_destroy(h)
            self._h = None

    def __del__(self):
        # fj_batch_destroy calls into the HIP runtime (it frees the recorded
        # graph); at interpreter shutdown that runtime may already be gone, so
        # the handle is left to the process's end there (late in shutdown the
        # module globals, sys among them, may already be None)
        try:
            if sys.is_finalizing():
                return
        except AttributeError:
            return
        self.close()


# ------------------------------------------------------------ learned warm start
def _net_lib():
    L = lib()
    if not getattr(L, "_net_ready", False):
        vp, i32, sz, fl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t, ctypes.c_float
        L.fj_wsnet_param_count.restype = i32
        L.fj_wsnet_workspace_bytes.argtypes = [vp, i32]
        L.fj_wsnet_workspace_bytes.restype = sz
        L.fj_wsnet_forward.argtypes = [vp, vp, vp, vp, vp, sz, vp]
        L.fj_wsnet_forward.restype = i32
        L.fj_wsnet_forward_timed.argtypes = [vp, vp, vp, vp, vp, sz, vp, vp]
        L.fj_wsnet_forward_timed.restype = i32
        L.fj_wsnet_grad.argtypes = [vp, vp, vp, vp, ctypes.c_double, vp, vp, vp, sz, vp]
        L.fj_wsnet_grad.restype = i32
        L.fj_wsnet_train_step.argtypes = [vp, vp, vp, vp, vp, vp, i32, fl, ctypes.c_double, vp, vp, sz, vp]
        L.fj_wsnet_train_step.restype = i32
        L.fj_jacobi_workspace_bytes.argtypes = [vp]
        L.fj_jacobi_workspace_bytes.restype = sz
        L.fj_jacobi_steps.argtypes = [vp, vp, vp, i32, vp, sz, vp]
        L.fj_jacobi_steps.restype = i32
        L._net_ready = True
    return L


def wsnet_param_count() -> int:
    return int(_net_lib().fj_wsnet_param_count())


def _net_ws(graph: Graph, training: bool) -> torch.Tensor:
    attr = "_net_ws_train" if training else "_net_ws_inf"
    nbytes = _net_lib().fj_wsnet_workspace_bytes(graph.handle, 1 if training else 0)
    ws = getattr(graph, attr, None)
    if ws is None or ws.numel() < nbytes:
        ws = _workspace(nbytes, graph.device)
        setattr(graph, attr, ws)
    return ws


def wsnet_forward(graph: Graph, s: torch.Tensor, params: torch.Tensor, out: Optional[torch.Tensor] = None):
    """Warm-start proposal z0 (FP64 [n]) from the network with FP32 params."""
    n = graph.n
    _dev_ptr(s, torch.float64, n, "s")
    _dev_ptr(params, torch.float32, wsnet_param_count(), "params")
    z0 = out if out is not None else torch.empty(n, dtype=torch.float64, device=graph.device)
    ws = _net_ws(graph, False)
    _check(_net_lib().fj_wsnet_forward(graph.handle, ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(params.data_ptr()),
                                       ctypes.c_void_p(z0.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                       _stream()))
    return z0


def wsnet_forward_timed(graph: Graph, s: torch.Tensor, params: torch.Tensor, out: Optional[torch.Tensor] = None):
    """wsnet_forward with its stages timed by HIP events: (z0, [ms of the
    gather of s, layer 1, the gather of P, layer 2])."""
    n = graph.n
    _dev_ptr(s, torch.float64, n, "s")
    _dev_ptr(params, torch.float32, wsnet_param_count(), "params")
    z0 = out if out is not None else torch.empty(n, dtype=torch.float64, device=graph.device)
    ws = _net_ws(graph, False)
    ms = (ctypes.c_double * 4)()
    _check(_net_lib().fj_wsnet_forward_timed(graph.handle, ctypes.c_void_p(s.data_ptr()),
                                             ctypes.c_void_p(params.data_ptr()), ctypes.c_void_p(z0.data_ptr()),
                                             ctypes.c_void_p(ws.data_ptr()), ws.numel(), ms, _stream()))
    return z0, [float(x) for x in ms]


def wsnet_grad(graph: Graph, s: torch.Tensor, z_target: torch.Tensor, params: torch.Tensor, rel_floor: float = 0.0):
    """(loss, grad) of the mean over nodes of w (z0 - z_target)^2, with
    w = 1 / (z_target + rel_floor)^2 when rel_floor > 0, else 1."""
    n = graph.n
    _dev_ptr(z_target, torch.float64, n, "z_target")
    grad = torch.empty(wsnet_param_count(), dtype=torch.float32, device=graph.device)
    loss = torch.empty(1, dtype=torch.float32, device=graph.device)
    ws = _net_ws(graph, True)
    _check(_net_lib().fj_wsnet_grad(graph.handle, ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(z_target.data_ptr()),
                                    ctypes.c_void_p(params.data_ptr()), float(rel_floor), ctypes.c_void_p(grad.data_ptr()),
                                    ctypes.c_void_p(loss.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                    _stream()))
    return loss, grad


def wsnet_train_step(graph: Graph, s: torch.Tensor, z_target: torch.Tensor, params: torch.Tensor,
                     m: torch.Tensor, v: torch.Tensor, step: int, lr: float, rel_floor: float = 0.0) -> torch.Tensor:
    """One Adam step in place on params (m, v: moment buffers).  Returns the
    loss (device scalar) of the forward pass before the step."""
    loss = torch.empty(1, dtype=torch.float32, device=graph.device)
    ws = _net_ws(graph, True)
    _check(_net_lib().fj_wsnet_train_step(graph.handle, ctypes.c_void_p(s.data_ptr()),
                                          ctypes.c_void_p(z_target.data_ptr()), ctypes.c_void_p(params.data_ptr()),
                                          ctypes.c_void_p(m.data_ptr()), ctypes.c_void_p(v.data_ptr()), int(step),
                                          float(lr), float(rel_floor), ctypes.c_void_p(loss.data_ptr()),
                                          ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return loss


def jacobi_steps(graph: Graph, s: torch.Tensor, z: torch.Tensor, steps: int) -> torch.Tensor:
    """In place: `steps` synchronous FJ updates (Eq. (1)) of z."""
    n = graph.n
    _dev_ptr(s, torch.float64, n, "s")
    _dev_ptr(z, torch.float64, n, "z")
    nbytes = _net_lib().fj_jacobi_workspace_bytes(graph.handle)
    ws = _workspace(nbytes, graph.device)
    _check(_net_lib().fj_jacobi_steps(graph.handle, ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(z.data_ptr()),
                                      int(steps), ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return z
