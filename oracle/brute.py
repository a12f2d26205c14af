"""ctypes wrapper of brute_count.c (oracle, test infrastructure only).

``build()`` compiles brute_count.c with gcc into oracle/_brute_count.so; the
functions here fail loudly if it is missing.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "brute_count.c")
LIB = os.path.join(_HERE, "_brute_count.so")
_lib = None


def build_brute(verbose: bool = False) -> str:
    """Compile brute_count.c (plain C, OpenMP) into _brute_count.so."""
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", LIB + ".tmp", SRC]
    subprocess.run(cmd, check=True, capture_output=not verbose)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(LIB)
        lib.oracle_level_histogram.argtypes = [ctypes.c_int, ctypes.c_int,
                                               ctypes.c_void_p, ctypes.c_void_p]
        lib.oracle_cost_range.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                          ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p]
        _lib = lib
    return _lib


def level_histogram_brute(n: int, lits) -> np.ndarray:
    """N_k for k = 0..m by brute force over all 2^n assignments."""
    lits = np.ascontiguousarray(np.asarray(lits, dtype=np.int32).reshape(-1, 3))
    m = lits.shape[0]
    hist = np.zeros(m + 1, dtype=np.uint64)
    rc = _load().oracle_level_histogram(n, m, lits.ctypes.data, hist.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_level_histogram: bad arguments")
    return hist.astype(np.int64)


def cost_range_brute(n: int, lits, z0: int, count: int) -> np.ndarray:
    """C(z) for z in [z0, z0 + count) by brute force (uint8)."""
    lits = np.ascontiguousarray(np.asarray(lits, dtype=np.int32).reshape(-1, 3))
    out = np.empty(count, dtype=np.uint8)
    rc = _load().oracle_cost_range(n, lits.shape[0], lits.ctypes.data, z0, count, out.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_cost_range: bad arguments")
    return out
