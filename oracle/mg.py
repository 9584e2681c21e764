"""Multigrid solve of the oracle's systems for grids too large to factor.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  A ctypes front end for
oracle/mg.c, a plain FP64 geometric multigrid: Galerkin coarse operators of
the piecewise-constant prolongation over 2^d aggregates, red-black
Gauss-Seidel, an exact dense coarsest solve, preconditioned conjugate
gradients, and iterative refinement with long-double flux-form residuals.
It solves the same operator as the direct solve (solve.FluxOp, through its
per-axis couplings ``plus``) to the discrete solution: the refinement stops
when a correction no longer changes x in double precision.

The library is built by build() (gcc -O3 -fopenmp); a missing library is an
error, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmgoracle.so")
SRC_PATH = os.path.join(_HERE, "mg.c")
_lib = None


def build(verbose=False):
    """Compile oracle/mg.c into oracle/libmgoracle.so (plain C, OpenMP)."""
    import subprocess
    cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-Wno-unknown-pragmas",
           SRC_PATH, "-o", LIB_PATH + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    global _lib
    _lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build()")
        lib = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.oracle_mg_solve.argtypes = [ctypes.c_int, ip, ip, dp, ctypes.POINTER(dp), dp, dp, ctypes.c_double,
                                        ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int, dp]
        lib.oracle_mg_solve.restype = ctypes.c_int
        _lib = lib
    return _lib


class MGError(RuntimeError):
    pass


def solve_op(op, b, rtol=1e-16, max_rounds=6, inner_rtol=1e-10, max_iters=500, nu=2, gamma=2,
             threads=0, info=None):
    """Solve op x = b for a solve.FluxOp carrying ``plus`` and ``shape``.

    Returns x (float64).  ``info`` (a dict, optional) receives the final
    relative residual of the returned x (long-double flux form), the
    refinement rounds, the PCG iterations and the number of levels."""
    if op.plus is None or op.shape is None:
        raise MGError("the operator carries no per-axis couplings")
    lib = _load()
    (n, per) = op.shape
    dim = len(op.plus)
    N = int(n[0]) * int(n[1]) * int(n[2])
    m = np.ascontiguousarray(op.mexc, dtype=np.float64)
    ws = [np.ascontiguousarray(op.plus[a], dtype=np.float64) for a in range(dim)]
    bb = np.ascontiguousarray(b, dtype=np.float64).ravel()
    if m.size != N or bb.size != N or any(w.size != N for w in ws):
        raise MGError("sizes do not match the grid")
    x = np.zeros(N)
    dp = ctypes.POINTER(ctypes.c_double)
    warr = (dp * 3)(*[w.ctypes.data_as(dp) for w in ws], *([None] * (3 - dim)))
    narr = (ctypes.c_int * 3)(*[int(v) for v in n])
    parr = (ctypes.c_int * 3)(*[int(bool(v)) for v in per])
    inf = np.zeros(8)
    rc = lib.oracle_mg_solve(dim, narr, parr, m.ctypes.data_as(dp), warr, bb.ctypes.data_as(dp),
                             x.ctypes.data_as(dp), rtol, max_rounds, inner_rtol, max_iters, nu, gamma,
                             int(threads), inf.ctypes.data_as(dp))
    if info is not None:
        info.update(rel_res=inf[0], rounds=int(inf[1]), pcg_iters=int(inf[2]), levels=int(inf[3]),
                    first_round_iters=int(inf[4]), last_correction=inf[5], rel_res_ld=inf[6])
    if rc not in (0, -3):
        raise MGError(f"oracle_mg_solve failed with code {rc}")
    return x


def solver(threads=0, **kw):
    """A solver with the signature of solve.direct (A is not used)."""
    def _solve(A, b, op=None):
        if op is None:
            raise MGError("the multigrid solve needs the flux-form operator")
        if not np.any(b):
            return np.zeros_like(b)
        return solve_op(op, b, threads=threads, **kw)
    return _solve
