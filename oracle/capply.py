"""Oracle: the completed double-layer operator applied in plain C (cdlp.c).

TEST INFRASTRUCTURE ONLY (tests, the script that writes stored reference
solutions, the CPU-baseline leg of the benchmark).  The C file is compiled by
gcc with OpenMP into ``oracle/_cdlp.so`` on first use (or by ``build()``).

``apply(geom, u)`` is A u in double precision, one target row at a time over
all sources in index order (same formulas as ``dlp.rows_of_matrix``);
``apply(geom, u, extended=True)`` evaluates the same formulas in x87 80-bit
arithmetic, for residuals far below |A| |u|.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cdlp.c")
LIB = os.path.join(HERE, "_cdlp.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile cdlp.c (gcc, OpenMP) into _cdlp.so."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + f".{os.getpid()}.tmp"
        subprocess.run(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", SRC, "-o", tmp, "-lm"],
                       check=True)
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        p = ctypes.c_void_p
        for name in ("oracle_apply_f64", "oracle_apply_f80"):
            fn = getattr(lib, name)
            fn.argtypes = [ctypes.c_int64, ctypes.c_int32] + [p] * 14
            fn.restype = None
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def apply(geom, u: np.ndarray, extended: bool = False) -> np.ndarray:
    """A @ u for the completed double-layer matrix of ``geom``."""
    lib = _load()
    n = geom.n_unknowns
    u = np.ascontiguousarray(u, dtype=np.float64)
    assert u.shape == (n,)
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in
            (geom.x, geom.y, geom.nx, geom.ny, geom.tx, geom.ty, geom.w, geom.kappa,
             geom.cx, geom.cy, geom.radius)]
    off = np.ascontiguousarray(geom.curve_off, dtype=np.int64)
    out = np.empty(n)
    fn = lib.oracle_apply_f80 if extended else lib.oracle_apply_f64
    fn(geom.n_nodes, geom.n_pores, _ptr(off), *[_ptr(a) for a in arrs], _ptr(u), _ptr(out))
    return out
