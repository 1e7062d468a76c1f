"""ctypes wrapper of the C PageRank oracle (oracle/cpr.c).

TEST INFRASTRUCTURE ONLY: used by tests for graphs too large for the numpy
oracle to finish in seconds (the 16M-vertex banded workload); never by the
product path.  It computes the same Jacobi iterates as
``oracle.pagerank.pagerank_jacobi`` (the per-vertex sums in the same edge
order), in parallel over vertices.  ``build()`` compiles the library with the
host C compiler; importing this module builds it when it is missing.
"""
from __future__ import annotations

import ctypes as C
import os
import shutil
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "cpr.c")
LIB = os.path.join(_HERE, "libcpr.so")


def build(verbose=False):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        raise RuntimeError("no host C compiler for the C oracle")
    cmd = [cc, "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", SRC, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, capture_output=not verbose)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def _load():
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    lib = C.CDLL(LIB)
    lib.cpr_jacobi.restype = C.c_int
    lib.cpr_jacobi.argtypes = [C.c_uint32, C.c_uint64, C.c_void_p, C.c_void_p, C.c_uint32, C.c_double, C.c_double,
                               C.c_uint32, C.c_void_p, C.POINTER(C.c_uint32), C.POINTER(C.c_double)]
    return lib


_lib = None


def pagerank_jacobi(g, alpha=0.85, tol=1e-6, max_sweeps=10_000, restart=None):
    """(x, sweeps, last L1 change) of synchronous PageRank from 1/N (or of
    personalised PageRank from e_restart), stopping after the first sweep
    whose L1 change is below tol (counted)."""
    global _lib
    if _lib is None:
        _lib = _load()
    ptr = np.ascontiguousarray(g.ptr, dtype=np.uint64)
    idx = np.ascontiguousarray(g.idx, dtype=np.uint32)
    x = np.empty(g.n, dtype=np.float64)
    sw, r = C.c_uint32(), C.c_double()
    rs = 0xFFFFFFFF if restart is None else int(restart)
    st = _lib.cpr_jacobi(g.n, idx.size, ptr.ctypes.data, idx.ctypes.data, rs, alpha, tol, max_sweeps, x.ctypes.data,
                         C.byref(sw), C.byref(r))
    if st != 0:
        raise ValueError(f"C oracle failed with status {st}")
    return x, int(sw.value), float(r.value)


def pagerank_fixed_point(g, alpha=0.85, tol=1e-12, max_sweeps=100_000):
    """x* as oracle.pagerank.pagerank_fixed_point: Jacobi to an L1 change
    below tol, then one normalisation."""
    x, _, _ = pagerank_jacobi(g, alpha, tol, max_sweeps)
    return x / x.sum()


def ppr_fixed_point(g, s, alpha=0.85, tol=1e-12, max_sweeps=100_000):
    """x*_s as oracle.pagerank.ppr_fixed_point."""
    x, _, _ = pagerank_jacobi(g, alpha, tol, max_sweeps, restart=s)
    return x / x.sum()
