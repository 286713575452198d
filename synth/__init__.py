"""Seeded synthetic inputs for the Friedkin-Johnsen solver: graphs and opinions.

Holds none of the method's arithmetic.  Both the FP64 oracle and the HIP
library are fed from here so that they see identical inputs.  The generators
are C (``synth.c``, built into ``libsynth.so`` by ``synth.build``); this module
only marshals numpy arrays.

Graph convention (Sec. 3.2-3.3): CSR of the adjacency matrix A, row i lists the
j with a_ij > 0, i.e. the nodes whose expressed opinion node i averages in the
FJ update, Eq. (1).  Rows are sorted, without self-loops or duplicates.
"""
import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

S_UNIFORM, S_BETA, S_BIMODAL, S_EXP, S_PARETO = 0, 1, 2, 3, 4


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "libsynth.so")
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(path)
        i64, u64, i32, dbl = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int, ctypes.c_double
        vp = ctypes.c_void_p
        lib.synth_opinions.argtypes = [i64, i32, i32, i32, dbl, u64, vp]
        lib.synth_opinions.restype = i32
        lib.synth_ba.argtypes = [i64, i32, u64, vp, vp, i64]
        lib.synth_ba.restype = i64
        lib.synth_chung_lu.argtypes = [i64, i64, dbl, dbl, i32, u64, vp, vp, i64, i32, dbl, dbl, vp]
        lib.synth_chung_lu.restype = i64
        _LIB = lib
    return _LIB


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class CSRGraph:
    """Host CSR graph.  ``w`` is None for unit weights."""
    n: int
    row_ptr: np.ndarray  # int32 [n+1]
    col: np.ndarray      # int32 [nnz]
    w: Optional[np.ndarray]  # float32 [nnz] or None
    directed: bool

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])


def opinions(n: int, kind: str = "uniform", seed: int = 0, a: int = 2, b: int = 8,
             p1: Optional[float] = None) -> np.ndarray:
    """Internal opinions s in [0,1] (FP64).

    kinds: ``uniform`` U[0,1]; ``beta`` Beta(a,b); ``bimodal``
    0.5 Beta(a,b) + 0.5 Beta(b,a); ``exp`` x_min + Exp(1) divided by the max
    (x_min = p1, default 1); ``pareto`` Pareto(alpha = p1, default 2.5) divided by
    the max.  The last three follow the opinion distributions of Sec. 6.
    """
    codes = {"uniform": S_UNIFORM, "beta": S_BETA, "bimodal": S_BIMODAL,
             "exp": S_EXP, "pareto": S_PARETO}
    if p1 is None:
        p1 = 2.5 if kind == "pareto" else 1.0
    s = np.empty(n, dtype=np.float64)
    rc = _lib().synth_opinions(n, codes[kind], a, b, float(p1), seed & (2**64 - 1), _ptr(s))
    if rc != 0:
        raise ValueError(f"synth_opinions failed for kind={kind} a={a} b={b}")
    return s


def barabasi_albert(n: int, m: int, seed: int) -> CSRGraph:
    """Undirected Barabasi-Albert graph with unit weights, stored both ways."""
    E = (m + 1) * m // 2 + (n - m - 1) * m
    row_ptr = np.empty(n + 1, dtype=np.int32)
    col = np.empty(2 * E, dtype=np.int32)
    nnz = _lib().synth_ba(n, m, seed, _ptr(row_ptr), _ptr(col), col.size)
    if nnz < 0:
        raise ValueError("synth_ba failed")
    return CSRGraph(n, row_ptr, col[:nnz].copy(), None, False)


def chung_lu(n: int, m: int, gamma: float, seed: int, directed: bool = False,
             weighted: bool = False, wlo: float = 0.5, whi: float = 1.5,
             wmax: float = 0.0) -> CSRGraph:
    """Chung-Lu power-law graph: ``m`` edge samples (undirected, stored both
    ways) or arc samples (directed), degree exponent ``gamma``, node 0
    heaviest.  Self-loops and duplicate samples are dropped."""
    slots = m if directed else 2 * m
    row_ptr = np.empty(n + 1, dtype=np.int32)
    col = np.empty(slots, dtype=np.int32)
    w = np.empty(slots, dtype=np.float32) if weighted else None
    nnz = _lib().synth_chung_lu(n, m, float(gamma), float(wmax), 0 if directed else 1, seed,
                                _ptr(row_ptr), _ptr(col), col.size, 1 if weighted else 0,
                                float(wlo), float(whi), _ptr(w) if weighted else None)
    if nnz < 0:
        raise ValueError("synth_chung_lu failed")
    col = col[:nnz]
    if w is not None:
        w = w[:nnz]
    return CSRGraph(n, row_ptr, col, w, directed)
