"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

The oracle and the input generators (plain C) are rebuilt with gcc's
-fsanitize=address,undefined and driven through their Python wrappers on
small graphs of every kind the tests use; the library's host code (argument
checks, workspace sizing, the batch layout) is rebuilt with the sanitizers on
its host pass only and called on its host-only paths.  Each run is a child
process with the sanitizer runtime preloaded, failing on the first report.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:protect_shadow_gap=0:abort_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}

ORACLE_DRIVER = r'''
import sys, numpy as np
sys.path.insert(0, ROOT)
import oracle, synth
from tests import graphs
oracle._HERE = LIBDIR; oracle._LIB = None
synth._HERE = LIBDIR; synth._LIB = None
cases = [synth.barabasi_albert(300, 3, 1), synth.chung_lu(2000, 12000, 2.3, 2),
         synth.chung_lu(1500, 9000, 2.1, 3, directed=True, weighted=True), graphs.random_graph(40, 0.2, 4),
         graphs.random_graph(1, 0.0, 5)]
for kind in ("uniform", "beta", "bimodal", "exp", "pareto"):
    synth.opinions(500, kind, 6)
for g in cases:
    s = synth.opinions(g.n, "bimodal", 7)
    zx = oracle.exact(g, s)
    for omega in ((1.0, 1.5) if not g.directed else (1.0,)):
        p = oracle.push(g, s, 1e-4, omega=omega)
        assert oracle.certificate(g, s, p["z"], 1e-4) <= 1.0 + 1e-9
    m = oracle.metrics(g, s, zx)
    oracle.transpose(g)
print("sanitized oracle clean", flush=True)
'''

HOST_DRIVER = r'''
import ctypes, sys
sys.path.insert(0, ROOT)
from paper_2507_14864_amd.fj import GraphDesc, MetricsOut, BatchItemDesc
L = ctypes.CDLL(LIBPATH)
L.fj_graph_workspace_bytes.argtypes = [ctypes.POINTER(GraphDesc), ctypes.c_int32]
L.fj_graph_workspace_bytes.restype = ctypes.c_size_t
dummy = ctypes.c_void_p(256)
for n, nnz, w, d in [(1000, 5000, None, 0), (1, 0, None, 0), (10**6, 10**7, dummy, 1), (-1, 5, None, 0), (0, 0, None, 0)]:
    desc = GraphDesc(n, nnz, dummy, dummy, w, d)
    for flags in (0, 1, 2):
        L.fj_graph_workspace_bytes(ctypes.byref(desc), flags)
L.fj_optimal_omega.argtypes = [ctypes.c_double]
L.fj_optimal_omega.restype = ctypes.c_double
for mu in (0.0, 0.5, 0.999, 1.0, -1.0, float("nan")):
    L.fj_optimal_omega(mu)
out = MetricsOut()
assert L.fj_metrics_noalloc(None, None, None, ctypes.byref(out), None) == 1
assert L.fj_solve(None, None, None, None, None, 0, None, None) == 1
L.fj_batch_workspace_bytes.argtypes = [ctypes.POINTER(BatchItemDesc), ctypes.c_int32]
L.fj_batch_workspace_bytes.restype = ctypes.c_size_t
items = (BatchItemDesc * 3)()
items[0].graph = GraphDesc(1000, 8000, dummy, dummy, None, 0); items[0].k = 1
items[1].graph = GraphDesc(5000, 40000, dummy, dummy, dummy, 1); items[1].k = 1
items[2].graph = GraphDesc(20000, 100000, dummy, dummy, None, 0); items[2].k = 64
assert L.fj_batch_workspace_bytes(items, 3) > 0
items[2].k = 65
assert L.fj_batch_workspace_bytes(items, 3) == 0
print("sanitized host code clean", flush=True)
'''


def _run(driver, preload, **subst):
    code = driver
    for k, v in subst.items():
        code = code.replace(k, repr(v))
    env = dict(os.environ, **SAN_ENV, LD_PRELOAD=preload)
    return subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)


def test_oracle_and_generators_under_asan_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if not gcc:
        pytest.skip("no gcc")
    flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
             "-fopenmp", "-fPIC", "-shared", "-std=c11", "-fno-fast-math"]
    for src, lib in (("oracle/fj_oracle.c", "liboracle.so"), ("synth/synth.c", "libsynth.so")):
        subprocess.run([gcc, *flags, os.path.join(ROOT, src), "-o", str(tmp_path / lib), "-lm"], check=True)
    asan = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    out = _run(ORACLE_DRIVER, asan, ROOT=ROOT, LIBDIR=str(tmp_path))
    assert out.returncode == 0 and "sanitized oracle clean" in out.stdout, out.stderr[-3000:]
    assert "runtime error" not in out.stderr


def test_library_host_code_under_asan_ubsan(tmp_path):
    hipcc = shutil.which("hipcc")
    if not hipcc:
        pytest.skip("no hipcc")
    from paper_2507_14864_amd import build as fjb
    csrc = os.path.join(ROOT, "paper_2507_14864_amd", "csrc")
    srcs = sorted(f for f in os.listdir(csrc) if f.endswith(".hip"))
    san = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    procs = []
    for f in srcs:
        cmd = [hipcc, *[x for x in fjb.hip_flags() if x != "-O3"], "-O1", "-g", *san, "-c", os.path.join(csrc, f),
               "-o", str(tmp_path / (f + ".o"))]
        procs.append(subprocess.Popen(cmd, stdout=subprocess.DEVNULL, stderr=subprocess.PIPE))
    for p in procs:
        _, err = p.communicate()
        assert p.returncode == 0, err.decode()[-2000:]
    lib = tmp_path / "libfj_san.so"
    subprocess.run([hipcc, f"--offload-arch={fjb.ARCH}", "-shared", "-fPIC", "-shared-libasan",
                    "-fsanitize=address,undefined", *[str(tmp_path / (f + ".o")) for f in srcs], "-o", str(lib)],
                   check=True, capture_output=True)
    rt = subprocess.run([hipcc, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                        text=True).stdout.strip()
    if not os.path.isabs(rt) or not os.path.exists(rt):
        pytest.skip("clang ASan runtime not found")
    out = _run(HOST_DRIVER, rt, ROOT=ROOT, LIBPATH=str(lib))
    assert out.returncode == 0 and "sanitized host code clean" in out.stdout, out.stderr[-3000:]
    assert "runtime error" not in out.stderr
