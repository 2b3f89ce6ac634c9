"""Loader of the C simulated-bifurcation oracle (``oracle/sb_omp.c``):
the steps of ``oracle.sb.run`` in FP64 C with the agents spread over host
threads (OpenMP).  Test infrastructure: only the tests and the benchmark's
CPU-baseline leg use it.  ``build()`` compiles it to
``oracle/libsboracle.so`` with gcc (-O2 -fopenmp -ffp-contract=off)."""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np
import scipy.sparse as sp

from .philox import initial_state

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sb_omp.c")
LIB = os.path.join(HERE, "libsboracle.so")
MODES = {"bsb": 0, "dsb": 1, "asb": 2}
_lib = None


def build() -> str:
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    "-fno-fast-math", "-std=c11", "-Wall", SRC, "-o", tmp], check=True)
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise ImportError(f"{LIB} is missing: build it with oracle.sb_c.build()")
        lib = C.CDLL(LIB)
        P = C.c_void_p
        lib.sbo_run.restype = C.c_int
        lib.sbo_run.argtypes = [C.c_int, P, P, P, P, C.c_double, C.c_int, C.c_int, C.c_int,
                                C.c_double, C.c_double, P, P, C.c_int, C.POINTER(C.c_int)]
        _lib = lib
    return _lib


def run(J: sp.csr_matrix, h, c0: float, mode: str, agents: int, steps: int, dt: float = 1.0,
        a0: float = 1.0, seed: int = 0, event: int = 0, x0=None, y0=None, threads: int = 0):
    """Final (x, y, threads used) of ``steps`` steps for ``agents`` shots;
    same arguments and start as ``oracle.sb.run``."""
    lib = _load()
    J = sp.csr_matrix(J, dtype=np.float64)
    J.sort_indices()
    n = int(np.asarray(h).shape[0])
    rp = np.ascontiguousarray(J.indptr, dtype=np.int64)
    col = np.ascontiguousarray(J.indices, dtype=np.int32)
    val = np.ascontiguousarray(J.data, dtype=np.float64)
    hh = np.ascontiguousarray(h, dtype=np.float64)
    if x0 is None or y0 is None:
        x0, y0 = initial_state(n, agents, seed, event)
    x = np.array(x0, dtype=np.float64, order="C", copy=True)
    y = np.array(y0, dtype=np.float64, order="C", copy=True)
    used = C.c_int(0)
    rc = lib.sbo_run(n, rp.ctypes.data, col.ctypes.data, val.ctypes.data, hh.ctypes.data,
                     float(c0), MODES[mode], int(agents), int(steps), float(dt), float(a0),
                     x.ctypes.data, y.ctypes.data, int(threads), C.byref(used))
    if rc != 0:
        raise RuntimeError("sbo_run failed")
    return x, y, used.value
