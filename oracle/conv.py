"""FP64 oracle of the 3x3 convolution layer (test infrastructure only).

The operation is the paper's Conv benchmark layer (Tiramisu paper, Section
VI-A: a direct convolution layer, here with a 3x3 filter) in the layout the
library takes: input X is NHWC (batch x H x W x Cin), the filter Wt is
3 x 3 x Cin x Cout, the output Y is NHWC (batch x H x W x Cout); stride 1 and
zero padding 1, so Y has the input's height and width:

  Y[n, y, x, co] = alpha * sum_{dy, dx, ci} Xpad[n, y + dy, x + dx, ci] * Wt[dy, dx, ci, co]
                   + beta * Y0[n, y, x, co]

where Xpad is X with one row and column of zeros on every side.  The sum is
taken over the nine taps, each a matrix product of the shifted input (as an
(n*H*W) x Cin matrix) with Wt[dy, dx] (a library matmul as a step), in FP64.
beta == 0 never reads Y0 (reference-BLAS reading).  Parity pinned by
tests/test_oracle.py (brute force, closed forms, explicit im2col + the gemm
oracle).
"""
import numpy as np


def _f64(x):
    if x is None:
        return None
    if hasattr(x, "detach"):
        x = x.detach().cpu().numpy()
    return np.asarray(x, dtype=np.float64)


def conv3x3(X, Wt, Y0=None, alpha=1.0, beta=0.0, pixels=None):
    """FP64 3x3 'same' convolution; returns batch x H x W x Cout.

    pixels: optional flat output-pixel indices (n*H*W + y*W + x); then only those
    rows of the (batch*H*W) x Cout result are computed and returned."""
    X = _f64(X)
    Wt = _f64(Wt)
    nb, H, W, cin = X.shape
    if Wt.shape[:3] != (3, 3, cin):
        raise ValueError(f"filter shape {Wt.shape} does not match input channels {cin}")
    cout = Wt.shape[3]
    Xp = np.zeros((nb, H + 2, W + 2, cin))
    Xp[:, 1:H + 1, 1:W + 1, :] = X
    if pixels is None:
        pix = np.arange(nb * H * W)
    else:
        pix = np.asarray(pixels, dtype=np.int64)
    n, rem = np.divmod(pix, H * W)
    y, x = np.divmod(rem, W)
    acc = np.zeros((len(pix), cout))
    for dy in range(3):
        for dx in range(3):
            acc += Xp[n, y + dy, x + dx, :] @ Wt[dy, dx]
    out = alpha * acc
    if beta != 0.0:
        out = out + beta * _f64(Y0).reshape(nb * H * W, cout)[pix]
    if pixels is None:
        return out.reshape(nb, H, W, cout)
    return out
