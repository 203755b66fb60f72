"""Multi-core FP64 twin of chebyshev.filter_recurrence (Sec. 2.2, Step 1; Sec. 3.2).

TEST INFRASTRUCTURE ONLY (see the package header).  oracle/cfilter.c computes
Y = sum_j a_j T_j(L~) X by the same three-term recurrence as the Python oracle, in plain C
with the rows of each product split among OpenMP threads; this module builds L~ with the
Python oracle and hands it over.  It serves the CPU baseline (the oracle timed on all host
cores) and the expected values of large cases.

Parity pins (tests/test_oracle_cfilter.py): equality with filter_recurrence to 1e-13
relative on normalized and combinatorial Laplacians, widths 1-7 and degrees 0-60, and the
same bits for 1 and 4 threads.

Build: compiled with gcc -O2 -fopenmp -ffp-contract=off (no fused multiply-adds, so each
operation rounds as the Python oracle's does) by oracle/build_c.py, which the package build
calls.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .operator import scaled_laplacian

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcsc_oracle.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python oracle/build_c.py`")
        lib = C.CDLL(LIB_PATH)
        lib.oracle_cheb_filter.restype = C.c_int
        lib.oracle_cheb_filter.argtypes = [C.c_int64, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                           C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]
        _lib = lib
    return _lib


def filter_recurrence_c(A, lmax: float, a: np.ndarray, X: np.ndarray, threads: int = 0,
                        Lt=None):
    """(Y, threads used): Y = sum_j a_j T_j(L~) X with L~ from A (or given as Lt)."""
    lib = _load()
    if Lt is None:
        Lt = scaled_laplacian(A, lmax)
    Lt = Lt.tocsr()
    X = np.ascontiguousarray(X, dtype=np.float64)
    if X.ndim == 1:
        X = X[:, None]
    n, w = X.shape
    rowptr = np.ascontiguousarray(Lt.indptr, dtype=np.int64)
    col = np.ascontiguousarray(Lt.indices, dtype=np.int32)
    val = np.ascontiguousarray(Lt.data, dtype=np.float64)
    a = np.ascontiguousarray(a, dtype=np.float64)
    Y = np.empty_like(X)
    used = lib.oracle_cheb_filter(n, w, rowptr.ctypes.data, col.ctypes.data, val.ctypes.data,
                                  len(a) - 1, a.ctypes.data, X.ctypes.data, Y.ctypes.data,
                                  int(threads))
    if used < 0:
        raise MemoryError("oracle_cheb_filter: out of memory")
    return Y, used
