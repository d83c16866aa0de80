"""ctypes front end of the FP64 gemm reference (gemm_ref.c).

Test infrastructure only (see the package docstring).

gemm(A, B, C0, alpha, beta) returns alpha*A@B + beta*C0 in float64, computed
by the plain i-k-j triple loop of gemm_ref.c (Tiramisu paper, Section I: the
gemm problem statement).  Inputs may be float32 or float64 arrays; float32
values convert to float64 exactly, so the oracle sees the stored bits.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(lib_path):
            from .build_oracle import build
            build()
        lib = ctypes.CDLL(lib_path)
        i64, dbl, p = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
        lib.oracle_gemm_f64.argtypes = [i64, i64, i64, dbl, p, i64, p, i64,
                                        dbl, p, i64, p, i64]
        lib.oracle_gemm_f64.restype = ctypes.c_int
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _as_f64(x):
    if x is None:
        return None
    if hasattr(x, "detach"):  # torch tensor on the CPU
        x = x.detach().cpu().numpy()
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def gemm(A, B, C0=None, alpha=1.0, beta=0.0):
    """FP64 alpha*A@B + beta*C0 with reference-BLAS degenerate cases.

    A is M x K, B is K x N, C0 is M x N (ignored when beta == 0).
    """
    A = _as_f64(A)
    B = _as_f64(B)
    M, K = A.shape
    K2, N = B.shape
    if K2 != K:
        raise ValueError(f"inner dimensions differ: {A.shape} @ {B.shape}")
    C = np.empty((M, N), dtype=np.float64)
    if beta != 0.0:
        C0 = _as_f64(C0)
        if C0.shape != (M, N):
            raise ValueError("C0 shape")
        c0p, ldc0 = C0.ctypes.data, N
    else:
        c0p, ldc0 = None, N
    rc = _load().oracle_gemm_f64(M, N, K, float(alpha),
                                 A.ctypes.data if A.size else None, max(K, 1),
                                 B.ctypes.data if B.size else None, max(N, 1),
                                 float(beta), c0p, max(ldc0, 1),
                                 C.ctypes.data if C.size else None, max(N, 1))
    if rc != 0:
        raise ValueError("oracle_gemm_f64 rejected its arguments")
    return C


def gemm_rows(A, B, C0, alpha, beta, rows):
    """Rows `rows` of alpha*A@B + beta*C0: the same triple loop on A[rows]."""
    rows = np.asarray(rows, dtype=np.int64)
    A = A[rows] if not hasattr(A, "index_select") else A[rows]
    c0 = None
    if beta != 0.0:
        c0 = C0[rows]
    return gemm(A, B, c0, alpha, beta)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def normwise_error(X, R) -> float:
    """Frobenius-norm relative error ||X - R||_F / ||R||_F, sums in FP64."""
    X = _as_f64(X)
    R = _as_f64(R)
    den = np.sqrt(np.sum(R * R))
    num = np.sqrt(np.sum((X - R) * (X - R)))
    if den == 0.0:
        return float(num)
    return float(num / den)
