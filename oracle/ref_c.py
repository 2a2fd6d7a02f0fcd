"""ctypes access to the plain C reference of the MPK (oracle/mpk_ref.c) --
TEST INFRASTRUCTURE ONLY (tests/, smoke() and bench.py's cpu_baseline leg).

``build()`` compiles it with gcc (-O2 -ffp-contract=off, OpenMP) into
oracle/libmpk_ref.so; ``mpk(A, x, p)`` and ``mpk_omp(A, x, p, threads)`` call it.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mpk_ref.c")
LIB = os.path.join(HERE, "libmpk_ref.so")
CFLAGS = ["-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c11"]

_lib = None


def build():
    """Compiles the reference (always, also when a library exists)."""
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", *CFLAGS, SRC, "-o", tmp], check=True)
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise ImportError(f"{LIB} is not built: run oracle.ref_c.build()")
        lib = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        lib.mpk_ref.argtypes = [ctypes.c_int32, P, P, P, P, P, ctypes.c_int32]
        lib.mpk_ref.restype = None
        lib.mpk_ref_omp.argtypes = [ctypes.c_int32, P, P, P, P, P, ctypes.c_int32, ctypes.c_int32]
        lib.mpk_ref_omp.restype = ctypes.c_int32
        _lib = lib
    return _lib


def _args(A, x, p):
    n, rowptr, col, val = A
    rp = np.ascontiguousarray(rowptr, dtype=np.int32)
    c = np.ascontiguousarray(col, dtype=np.int32)
    v = np.ascontiguousarray(val, dtype=np.float64)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    Y = np.empty((int(p), int(n)), dtype=np.float64)
    return int(n), rp, c, v, xx, Y


def mpk(A, x, p):
    """(p, n) array of A^k x, k = 1..p, one thread."""
    lib = _load()
    n, rp, c, v, xx, Y = _args(A, x, p)
    lib.mpk_ref(n, rp.ctypes.data, c.ctypes.data, v.ctypes.data, xx.ctypes.data, Y.ctypes.data, int(p))
    return Y


def mpk_omp(A, x, p, threads=0):
    """(Y, threads used): the same powers with rows split over OpenMP threads."""
    lib = _load()
    n, rp, c, v, xx, Y = _args(A, x, p)
    used = lib.mpk_ref_omp(n, rp.ctypes.data, c.ctypes.data, v.ctypes.data, xx.ctypes.data, Y.ctypes.data,
                           int(p), int(threads))
    return Y, int(used)
