"""CPU oracle for the FastSimilarityGraph hot path (ctypes over libfsgo.so).

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the tests, the smoke
check and the benchmark's CPU-baseline leg import this module.  It shares
no code with the GPU library; see fsgo.h for the conventions it follows.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None
_I32P = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_I64P = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_F32P = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_F64P = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def _opt(ptr_type):
    """ndpointer that also accepts None (NULL)."""

    class _Opt(ptr_type):
        @classmethod
        def from_param(cls, obj):
            if obj is None:
                return None
            return ptr_type.from_param(obj)

    return _Opt


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        c_i64, c_i32, c_u64, c_dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double
        L.fsgo_philox4x64_10.argtypes = [np.ctypeslib.ndpointer(np.uint64), np.ctypeslib.ndpointer(np.uint64),
                                         np.ctypeslib.ndpointer(np.uint64)]
        L.fsgo_philox4x64_10.restype = None
        L.fsgo_philox_batch.argtypes = [np.ctypeslib.ndpointer(np.uint64), c_i64, np.ctypeslib.ndpointer(np.uint64),
                                        np.ctypeslib.ndpointer(np.uint64)]
        L.fsgo_philox_batch.restype = None
        L.fsgo_uniform.argtypes = [c_u64, c_u64, c_u64, ctypes.c_uint32]
        L.fsgo_uniform.restype = c_dbl
        L.fsgo_split.argtypes = [c_i64, c_i64]
        L.fsgo_split.restype = c_i64
        L.fsgo_kernel.argtypes = [_F32P, _F32P, c_i32, c_i32, c_dbl]
        L.fsgo_kernel.restype = c_dbl
        L.fsgo_degrees.argtypes = [_F32P, c_i64, c_i32, c_i32, c_dbl, _F64P]
        L.fsgo_degrees.restype = ctypes.c_int
        L.fsgo_kde_segmented.argtypes = [_F32P, c_i64, _F32P, c_i64, c_i32, c_i32, c_dbl, c_i64, _I64P, _I32P,
                                         _I32P, _I32P, _I32P, _opt(_I32P), _F64P, _F64P]
        L.fsgo_kde_segmented.restype = ctypes.c_int
        L.fsgo_sample_rows.argtypes = [_F32P, c_i64, c_i32, c_i32, c_dbl, c_i32, c_u64, _opt(_I32P), c_i64, _I32P,
                                       _opt(_F64P), _opt(_F64P)]
        L.fsgo_sample_rows.restype = ctypes.c_int
        L.fsgo_path_probability.argtypes = [_F32P, c_i64, c_i32, c_i32, c_dbl, c_i64, c_i64,
                                            ctypes.POINTER(ctypes.c_double)]
        L.fsgo_path_probability.restype = ctypes.c_int
        L.fsgo_build_csr.argtypes = [_F32P, c_i64, c_i32, c_i32, c_dbl, c_i32, _I32P, _opt(_F64P), _I64P, _I32P,
                                     _F64P, c_i64, ctypes.POINTER(ctypes.c_int64)]
        L.fsgo_build_csr.restype = ctypes.c_int
        L.fsgo_num_threads.argtypes = []
        L.fsgo_num_threads.restype = ctypes.c_int
        _LIB = L
    return _LIB


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def _points(X):
    X = np.ascontiguousarray(X, dtype=np.float32)
    if X.ndim != 2:
        raise ValueError("points must be a 2-D array")
    return X


def num_threads() -> int:
    return int(lib().fsgo_num_threads())


def philox4x64_10(ctr, key):
    ctr = np.ascontiguousarray(ctr, dtype=np.uint64)
    key = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().fsgo_philox4x64_10(ctr, key, out)
    return out


def philox_batch(ctrs, key):
    ctrs = np.ascontiguousarray(ctrs, dtype=np.uint64).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros_like(ctrs)
    lib().fsgo_philox_batch(ctrs, ctrs.shape[0], key, out)
    return out


def uniform(seed: int, i: int, l: int, level: int) -> float:
    return float(lib().fsgo_uniform(seed, i, l, level))


def split(a: int, b: int) -> int:
    return int(lib().fsgo_split(a, b))


# kernel kinds of Section 2.1 (the exponent holds ||x-y||_2^2, ||x-y||_2 or ||x-y||_1)
KERNELS = {"gaussian": 0, "exponential": 1, "laplacian": 2}


def _kind(kernel) -> int:
    return KERNELS[kernel] if isinstance(kernel, str) else int(kernel)


def kernel(x, y, gamma: float, kernel="gaussian") -> float:
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    return float(lib().fsgo_kernel(x, y, x.shape[0], _kind(kernel), gamma))


def degrees(X, gamma: float, kernel="gaussian"):
    X = _points(X)
    deg = np.zeros(X.shape[0], dtype=np.float64)
    _check(lib().fsgo_degrees(X, X.shape[0], X.shape[1], _kind(kernel), gamma, deg), "degrees")
    return deg


def kde_segmented(Q, X, gamma, q_ptr, q_idx, lo, mid, hi, self_idx=None, kernel="gaussian"):
    Q = _points(Q)
    X = _points(X)
    q_ptr = np.ascontiguousarray(q_ptr, dtype=np.int64)
    q_idx = np.ascontiguousarray(q_idx, dtype=np.int32)
    lo = np.ascontiguousarray(lo, dtype=np.int32)
    mid = np.ascontiguousarray(mid, dtype=np.int32)
    hi = np.ascontiguousarray(hi, dtype=np.int32)
    if self_idx is not None:
        self_idx = np.ascontiguousarray(self_idx, dtype=np.int32)
    n_seg = lo.shape[0]
    n_ent = int(q_ptr[-1]) if n_seg > 0 else 0
    left = np.zeros(max(n_ent, 1), dtype=np.float64)
    right = np.zeros(max(n_ent, 1), dtype=np.float64)
    _check(lib().fsgo_kde_segmented(Q, Q.shape[0], X, X.shape[0], X.shape[1], _kind(kernel), gamma, n_seg, q_ptr, q_idx,
                                    lo, mid, hi, self_idx, left, right), "kde_segmented")
    return left[:n_ent], right[:n_ent]


def sample_rows(X, gamma, L, seed, rows=None, want_margin=True, kernel="gaussian"):
    """Returns (nbr[n_rows, L], deg[n_rows], margin[n_rows, L] or None)."""
    X = _points(X)
    n = X.shape[0]
    if rows is not None:
        rows = np.ascontiguousarray(rows, dtype=np.int32)
        n_rows = rows.shape[0]
    else:
        n_rows = n
    nbr = np.zeros(max(n_rows * L, 1), dtype=np.int32)
    deg = np.zeros(max(n_rows, 1), dtype=np.float64)
    margin = np.zeros(max(n_rows * L, 1), dtype=np.float64) if want_margin else None
    _check(lib().fsgo_sample_rows(X, n, X.shape[1], _kind(kernel), gamma, L, seed, rows, n_rows, nbr, deg, margin),
           "sample_rows")
    nbr = nbr[: n_rows * L].reshape(n_rows, L)
    margin = margin[: n_rows * L].reshape(n_rows, L) if want_margin else None
    return nbr, deg[:n_rows], margin


def path_probability(X, gamma, i, j, kernel="gaussian") -> float:
    X = _points(X)
    p = ctypes.c_double(0.0)
    _check(lib().fsgo_path_probability(X, X.shape[0], X.shape[1], _kind(kernel), gamma, i, j, ctypes.byref(p)),
           "path_probability")
    return p.value


def build_csr(X, gamma, L, nbr, deg=None, kernel="gaussian"):
    """Returns (row_ptr int64[n+1], col int32[nnz], w float64[nnz])."""
    X = _points(X)
    n = X.shape[0]
    nbr = np.ascontiguousarray(nbr, dtype=np.int32).reshape(-1)
    if deg is not None:
        deg = np.ascontiguousarray(deg, dtype=np.float64)
    cap = 2 * n * L
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    col = np.zeros(max(cap, 1), dtype=np.int32)
    w = np.zeros(max(cap, 1), dtype=np.float64)
    nnz = ctypes.c_int64(0)
    _check(lib().fsgo_build_csr(X, n, X.shape[1], _kind(kernel), gamma, L, nbr, deg, row_ptr, col, w, cap,
                                ctypes.byref(nnz)),
           "build_csr")
    return row_ptr, col[: nnz.value].copy(), w[: nnz.value].copy()
