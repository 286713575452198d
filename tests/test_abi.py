"""The C-ABI library loads and exports every entry point include/fj.h declares.

No compute call is made here (no GPU in this tier); only the pure host
workspace-size query is exercised.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fj.h")
LIB = os.path.join(ROOT, "paper_2507_14864_amd", "libfj.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(fj_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2507_14864_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["fj_graph_create", "fj_solve", "fj_metrics", "fj_graph_destroy",
                     "fj_solve_workspace_bytes", "fj_graph_workspace_bytes", "fj_last_error"]:
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_graph_workspace_query_is_host_only(lib):
    from paper_2507_14864_amd.fj import GraphDesc
    f = lib.fj_graph_workspace_bytes
    f.argtypes = [ctypes.POINTER(GraphDesc), ctypes.c_int32]
    f.restype = ctypes.c_size_t
    dummy = ctypes.c_void_p(256)
    d = GraphDesc(1000, 5000, dummy, dummy, None, 0)
    plain = f(ctypes.byref(d), 0)
    coloured = f(ctypes.byref(d), 1)
    d2 = GraphDesc(1000, 5000, dummy, dummy, dummy, 1)
    directed = f(ctypes.byref(d2), 0)
    assert 0 < plain < coloured
    assert directed > plain  # CSR(A^T) with weights
    bad = GraphDesc(-1, 5, dummy, dummy, None, 0)
    assert f(ctypes.byref(bad), 0) == 0
    assert lib.fj_version() == 1


def test_binding_refuses_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    import paper_2507_14864_amd as fj
    with pytest.raises((RuntimeError, ValueError)):
        fj.Graph(torch.zeros(3, dtype=torch.int32), torch.zeros(0, dtype=torch.int32))


def test_optimal_omega_is_host_arithmetic(lib):
    """fj_optimal_omega is pure host code: Eq. (optimal-omega) against the oracle."""
    import oracle
    f = lib.fj_optimal_omega
    f.argtypes = [ctypes.c_double]
    f.restype = ctypes.c_double
    for mu in (0.0, 0.25, 2.0 / 3.0, 0.95, 0.999):
        assert abs(f(mu) - oracle.optimal_omega(mu)) <= 1e-15
    assert f(-1.0) == 1.0 and f(1.0) == 2.0 and f(float("nan")) == 1.0


def test_noalloc_metrics_host_checks(lib):
    """The allocation-free measures state their static size and reject a null
    graph before any device call."""
    from paper_2507_14864_amd.fj import MetricsOut
    lib.fj_metrics_noalloc_max_bytes.restype = ctypes.c_size_t
    assert lib.fj_metrics_noalloc_max_bytes() == 8 << 20
    lib.fj_metrics_noalloc_bytes.argtypes = [ctypes.c_void_p]
    lib.fj_metrics_noalloc_bytes.restype = ctypes.c_size_t
    assert lib.fj_metrics_noalloc_bytes(None) == 0
    f = lib.fj_metrics_noalloc
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(MetricsOut), ctypes.c_void_p]
    f.restype = ctypes.c_int32
    out = MetricsOut()
    assert f(None, None, None, ctypes.byref(out), None) == 1


def test_null_handles_are_rejected_on_the_host(lib):
    """Entry points added for tuning and measurement reject a null handle or
    out-of-range launch parameters with FJ_ERR_INVALID_ARGUMENT (1) before
    any device call."""
    vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    lib.fj_batch_set_launch.argtypes = [vp, i32, i32]
    lib.fj_batch_set_launch.restype = i32
    for nch, mu in ((4, 8), (3, 8), (4, 5), (16, 8)):
        assert lib.fj_batch_set_launch(None, nch, mu) == 1
    lib.fj_wsnet_forward_timed.argtypes = [vp, vp, vp, vp, vp, sz, vp, vp]
    lib.fj_wsnet_forward_timed.restype = i32
    ms = (ctypes.c_double * 4)()
    assert lib.fj_wsnet_forward_timed(None, None, None, None, None, 0, ms, None) == 1
    lib.fj_batch_set_omegas.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_double]
    lib.fj_batch_set_omegas.restype = i32
    assert lib.fj_batch_set_omegas(None, 1.0, 1.0, 1.0) == 1
