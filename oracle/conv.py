"""FP64 oracle of the convolution layer (test infrastructure only).

The operation is the paper's Conv benchmark layer (Tiramisu paper, Section
VI-A: a direct convolution layer with an R x R filter, R odd; the paper
names 3, 5, 7, 9 and 11) in the layout the library takes: input X is NHWC
(batch x H x W x Cin), the filter Wt is R x R x Cin x Cout, the output Y is
NHWC (batch x H x W x Cout); stride 1 and zero padding P = (R - 1) / 2, so Y
has the input's height and width:

  Y[n, y, x, co] = alpha * sum_{dy, dx, ci} Xpad[n, y + dy, x + dx, ci] * Wt[dy, dx, ci, co]
                   + beta * Y0[n, y, x, co]

where Xpad is X with P rows and columns of zeros on every side.  The sum is
taken over the R*R taps, each a matrix product of the shifted input (as an
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


def conv2d(X, Wt, Y0=None, alpha=1.0, beta=0.0, pixels=None):
    """FP64 R x R 'same' convolution (R = Wt.shape[0], odd); returns batch x H x W x Cout.

    pixels: optional flat output-pixel indices (n*H*W + y*W + x); then only those
    rows of the (batch*H*W) x Cout result are computed and returned."""
    X = _f64(X)
    Wt = _f64(Wt)
    nb, H, W, cin = X.shape
    R = Wt.shape[0]
    if R % 2 != 1 or Wt.shape[:3] != (R, R, cin):
        raise ValueError(f"filter shape {Wt.shape} is not R x R x {cin} with R odd")
    P = (R - 1) // 2
    cout = Wt.shape[3]
    Xp = np.zeros((nb, H + 2 * P, W + 2 * P, cin))
    Xp[:, P:H + P, P:W + P, :] = X
    if pixels is None:
        pix = np.arange(nb * H * W)
    else:
        pix = np.asarray(pixels, dtype=np.int64)
    n, rem = np.divmod(pix, H * W)
    y, x = np.divmod(rem, W)
    acc = np.zeros((len(pix), cout))
    for dy in range(R):
        for dx in range(R):
            acc += Xp[n, y + dy, x + dx, :] @ Wt[dy, dx]
    out = alpha * acc
    if beta != 0.0:
        out = out + beta * _f64(Y0).reshape(nb * H * W, cout)[pix]
    if pixels is None:
        return out.reshape(nb, H, W, cout)
    return out


def conv3x3(X, Wt, Y0=None, alpha=1.0, beta=0.0, pixels=None):
    """The 3 x 3 case of conv2d (filter 3 x 3 x Cin x Cout)."""
    if _f64(Wt).shape[:2] != (3, 3):
        raise ValueError("conv3x3 takes a 3 x 3 filter")
    return conv2d(X, Wt, Y0, alpha, beta, pixels)
