"""FP64 oracle of the binary tensor contraction (test infrastructure only).

The operation is the core of the paper's Baryon benchmark (Tiramisu paper,
Section VI-A: a dense tensor contraction), in the form the library takes:
dense row-major tensors whose modes carry integer labels, and

  C[modes_c] = alpha * sum over the modes of A and B absent from C of
               A[modes_a] * B[modes_b]  +  beta * C0[modes_c]

A mode in A, B and C is a batch mode, in A and C only a row (M) mode, in B and
C only a column (N) mode, in A and B only a contracted mode.  The sum is one
numpy.einsum call in FP64 (a library routine as the step; the labels become
einsum letters).  beta == 0 never reads C0 (reference-BLAS reading).  Parity
pinned by tests/test_oracle.py (brute force, the gemm oracle for the matrix
and batched-matrix cases, a transpose of the result by relabelling).
"""
import string

import numpy as np


def _f64(x):
    if x is None:
        return None
    if hasattr(x, "detach"):
        x = x.detach().cpu().numpy()
    return np.asarray(x, dtype=np.float64)


def contract(A, modes_a, B, modes_b, modes_c, C0=None, alpha=1.0, beta=0.0):
    """FP64 contraction; returns the tensor with modes `modes_c`."""
    A, B = _f64(A), _f64(B)
    labels = sorted(set(modes_a) | set(modes_b) | set(modes_c))
    if len(labels) > len(string.ascii_letters):
        raise ValueError("too many modes")
    letter = {m: string.ascii_letters[i] for i, m in enumerate(labels)}
    for modes, t in ((modes_a, A), (modes_b, B)):
        if len(modes) != t.ndim or len(set(modes)) != len(modes):
            raise ValueError("modes do not match the tensor")
    for m in modes_c:
        if m not in modes_a and m not in modes_b:
            raise ValueError(f"mode {m} of C is in neither operand")
    spec = "".join(letter[m] for m in modes_a) + "," + "".join(letter[m] for m in modes_b) + "->" + \
        "".join(letter[m] for m in modes_c)
    out = alpha * np.einsum(spec, A, B)
    if beta != 0.0:
        out = out + beta * _f64(C0)
    return out
