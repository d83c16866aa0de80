"""FP64 oracle of the back-to-back gemm (test infrastructure only).

The operation is the layer pair of the paper's VGG block (Tiramisu paper,
Section VI-A: two layers whose loops the compiler fuses so the intermediate
stays close to the arithmetic), written as two matrix products:

  T = act(A B)                 A: M x K, B: K x N1, T: M x N1
  E = alpha * T D + beta * E0  D: N1 x N2, E0 and E: M x N2

act is the identity or ReLU, max(x, 0) elementwise (NaN stays NaN).  Both
products are library matmuls in FP64 (steps of the definition, no blocking);
beta == 0 never reads E0 (reference-BLAS reading).  Parity pinned by
tests/test_oracle.py (brute force, the identity filter, composition through
the gemm oracle, closed forms).
"""
import numpy as np


def _f64(x):
    if x is None:
        return None
    if hasattr(x, "detach"):
        x = x.detach().cpu().numpy()
    return np.asarray(x, dtype=np.float64)


def gemm2(A, B, D, E0=None, alpha=1.0, beta=0.0, relu=False, rows=None):
    """FP64 alpha * act(A B) D + beta * E0; returns M x N2 (or the given rows)."""
    A, B, D = _f64(A), _f64(B), _f64(D)
    if A.shape[1] != B.shape[0] or B.shape[1] != D.shape[0]:
        raise ValueError(f"shapes do not chain: {A.shape} {B.shape} {D.shape}")
    r = np.arange(A.shape[0]) if rows is None else np.asarray(rows, dtype=np.int64)
    T = A[r] @ B
    if relu:
        T = np.where(T < 0.0, 0.0, T)   # max(x, 0) with NaN kept
    E = alpha * (T @ D)
    if beta != 0.0:
        E = E + beta * _f64(E0)[r]
    return E
