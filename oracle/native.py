"""ctypes wrapper of the oracle's plain C helpers (oracle/csrc/spm_oracle.c).

Test infrastructure only.  ``build()`` compiles the C file with gcc.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "spm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build() -> str:
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-o", _LIB, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        L.oracle_transpose_positions.argtypes = [i64, P, P, P]
        L.oracle_transpose_positions.restype = i64
        L.oracle_masked_product.argtypes = [i64, P, P, P, P, P]
        L.oracle_masked_product.restype = None
        L.oracle_masked_product_rows.argtypes = [i64, P, P, P, P, P, P]
        L.oracle_masked_product_rows.restype = i64
        L.oracle_masked_product_entries.argtypes = [i64, P, P, P, P, P, P, P, P, P]
        L.oracle_masked_product_entries.restype = None
        L.oracle_kernel_apply.argtypes = [i64, ctypes.c_int, P, i64, P, P, ctypes.c_int,
                                          ctypes.c_double, ctypes.c_double, ctypes.c_int, P]
        L.oracle_kernel_apply.restype = None
        L.oracle_kernel_apply_multi.argtypes = [i64, ctypes.c_int, P, i64, P, P, ctypes.c_int, ctypes.c_int,
                                                ctypes.c_double, ctypes.c_double, ctypes.c_int, P]
        L.oracle_kernel_apply_multi.restype = None
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_set_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def set_threads(n: int) -> int:
    """Sets the OpenMP thread count of the C helpers; returns the count a parallel region uses."""
    return int(lib().oracle_set_threads(int(n)))


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def transpose_positions(rp: np.ndarray, col: np.ndarray) -> np.ndarray:
    rp = np.ascontiguousarray(rp, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    tpos = np.empty(col.shape[0], dtype=np.int64)
    missing = lib().oracle_transpose_positions(rp.shape[0] - 1, _p(rp), _p(col), _p(tpos))
    if missing:
        raise ValueError("pattern is not structurally symmetric")
    return tpos


def masked_product_csr(rp, col, a, b, tpos=None) -> np.ndarray:
    """C = P_S(A B) for A, B stored on the same symmetric CSR pattern."""
    rp = np.ascontiguousarray(rp, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    if tpos is None:
        tpos = transpose_positions(rp, col)
    a = np.ascontiguousarray(a, dtype=np.float64)
    bt = np.ascontiguousarray(np.asarray(b, dtype=np.float64)[tpos])
    c = np.empty_like(a)
    lib().oracle_masked_product(rp.shape[0] - 1, _p(rp), _p(col), _p(a), _p(bt), _p(c))
    return c


def masked_product_rows(rows, rp, col, a, b, tpos=None):
    """Entries of P_S(A B) on the given rows; returns (values at those rows' positions, count)."""
    rp = np.ascontiguousarray(rp, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    if tpos is None:
        tpos = transpose_positions(rp, col)
    a = np.ascontiguousarray(a, dtype=np.float64)
    bt = np.ascontiguousarray(np.asarray(b, dtype=np.float64)[tpos])
    c = np.zeros_like(a)
    cnt = lib().oracle_masked_product_rows(rows.shape[0], _p(rows), _p(rp), _p(col), _p(a), _p(bt), _p(c))
    return c, int(cnt)


def masked_product_rows_bt(rows, rp, col, a, bt):
    """Entries of P_S(A B) on the given rows with B^T given directly on the pattern
    (bt[pos(j, k)] = b_kj); rows not needed may be empty in rp.  Returns (c, count)."""
    rp = np.ascontiguousarray(rp, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    a = np.ascontiguousarray(a, dtype=np.float64)
    bt = np.ascontiguousarray(bt, dtype=np.float64)
    c = np.zeros_like(a)
    cnt = lib().oracle_masked_product_rows(rows.shape[0], _p(rows), _p(rp), _p(col), _p(a), _p(bt), _p(c))
    return c, int(cnt)


def masked_product_entries(ii, jj, pos, rp, col, a, bt, c):
    """Entries c_ij of P_S(A B) at the listed (i, j) (written to c[pos]); bt holds B^T
    on the pattern (bt[pos(j, k)] = b_kj).  Returns the number of multiply-adds."""
    ii = np.ascontiguousarray(ii, dtype=np.int64)
    jj = np.ascontiguousarray(jj, dtype=np.int64)
    pos = np.ascontiguousarray(pos, dtype=np.int64)
    rp = np.ascontiguousarray(rp, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    a = np.ascontiguousarray(a, dtype=np.float64)
    bt = np.ascontiguousarray(bt, dtype=np.float64)
    assert c.dtype == np.float64 and c.flags.c_contiguous
    m = ctypes.c_int64(0)
    lib().oracle_masked_product_entries(ii.shape[0], _p(ii), _p(jj), _p(pos), _p(rp), _p(col), _p(a), _p(bt), _p(c),
                                        ctypes.byref(m))
    return int(m.value)


def kernel_apply(x: np.ndarray, y: np.ndarray, w: np.ndarray, p: int, ell: float, scale: float,
                 deriv: bool = False) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    out = np.empty(x.shape[0])
    lib().oracle_kernel_apply(x.shape[0], x.shape[1], _p(x), y.shape[0], _p(y), _p(w), p, ell, scale,
                              int(deriv), _p(out))
    return out


def kernel_apply_multi(x: np.ndarray, y: np.ndarray, w: np.ndarray, p: int, ell: float, scale: float,
                       deriv: bool = False) -> np.ndarray:
    """kernel_apply for the columns of w (m x k) at once; returns (n x k), each column
    bit-identical to kernel_apply with that column."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    k = w.shape[1]
    out = np.empty((x.shape[0], k))
    lib().oracle_kernel_apply_multi(x.shape[0], x.shape[1], _p(x), y.shape[0], _p(y), _p(w), k, p, ell, scale,
                                    int(deriv), _p(out))
    return out
