"""Seeded synthetic inputs for the gemm library and its tests.

This module only draws numbers; it holds none of the gemm arithmetic, so both
the GPU path and the oracle may use it.  Everything is generated on the CPU
(torch.Generator / numpy default_rng), so a GPU run and an oracle run see the
same bits.

Workloads (the paper's sgemm uses synthetic 1060 x 1060 single-precision
matrices, Section VI-A; no dataset is involved anywhere):
  gemm_inputs        A, B, C0 ~ U[-1, 1] float32, drawn in the order A, B, C0.
  lowprec_inputs     A, B ~ N(0, 1) float32 with 1% of the rows of A and 1%
                     of the rows of B (count max(1, round(0.01 rows)), chosen
                     by a seeded permutation) multiplied by exactly 1e3.
  integer_inputs     small integers in [-r, r] stored as float32.
  grouped_dims       d = rint(exp(U(ln lo, ln hi))) clipped to [lo, hi].
  conv_shapes        im2col shapes of 3x3 convolutions, batch 32:
                     M = 32 H W, N = Cout, K = 9 Cin.
"""
import math

import numpy as np
import torch


def _gen(seed):
    g = torch.Generator(device="cpu")
    g.manual_seed(int(seed))
    return g


def uniform(rows, cols, g):
    """U[-1, 1] as 2*rand - 1 in float32."""
    return 2.0 * torch.rand(rows, cols, generator=g, dtype=torch.float32) - 1.0


def gemm_inputs(M, N, K, seed):
    g = _gen(seed)
    A = uniform(M, K, g)
    B = uniform(K, N, g)
    C0 = uniform(M, N, g)
    return A, B, C0


def padded(X, extra_cols, fill=float("nan")):
    """X inside a wider row-major buffer: returns (buffer, leading dimension)."""
    rows, cols = X.shape
    buf = torch.full((rows, cols + extra_cols), fill, dtype=X.dtype)
    buf[:, :cols] = X
    return buf, cols + extra_cols


def integer_inputs(M, N, K, seed, r=8):
    g = _gen(seed)
    A = torch.randint(-r, r + 1, (M, K), generator=g).to(torch.float32)
    B = torch.randint(-r, r + 1, (K, N), generator=g).to(torch.float32)
    C0 = torch.randint(-r, r + 1, (M, N), generator=g).to(torch.float32)
    return A, B, C0


def _outlier_rows(rows, g):
    count = max(1, int(round(0.01 * rows)))
    return torch.randperm(rows, generator=g)[:count]


def lowprec_inputs(M, N, K, seed, factor=1e3):
    """A (M x K), B (K x N) ~ N(0,1) with 1% of the rows of each times 1e3."""
    g = _gen(seed)
    A = torch.randn(M, K, generator=g, dtype=torch.float32)
    B = torch.randn(K, N, generator=g, dtype=torch.float32)
    ra = _outlier_rows(M, g)
    rb = _outlier_rows(K, g)
    A[ra] *= factor
    B[rb] *= factor
    return A, B


def loguniform_dims(count, lo, hi, seed, width=3):
    rng = np.random.default_rng(seed)
    d = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=(count, width))))
    return np.clip(d, lo, hi).astype(np.int64)


def grouped_dims(count=512, lo=16, hi=2048, seed=4):
    """(count, 3) array of (M, N, K), log-uniform in [lo, hi]."""
    return loguniform_dims(count, lo, hi, seed)


def grouped_inputs(dims, seed_base=4000):
    """Per-problem (A, B, C0) ~ U[-1, 1], problem p drawn from seed_base + p."""
    out = []
    for p, (m, n, k) in enumerate(dims):
        out.append(gemm_inputs(int(m), int(n), int(k), seed_base + p))
    return out


def conv_layer_inputs(batch, H, W, cin, cout, seed, R=3):
    """X (batch, H, W, cin), Wt (R, R, cin, cout), Y0 (batch, H, W, cout), U[-1, 1] float32,
    drawn in that order from one seeded generator."""
    g = _gen(seed)
    X = uniform(batch * H * W, cin, g).reshape(batch, H, W, cin)
    Wt = uniform(R * R * cin, cout, g).reshape(R, R, cin, cout)
    Y0 = uniform(batch * H * W, cout, g).reshape(batch, H, W, cout)
    return X, Wt, Y0


def conv_shapes(batch=32, spatial=(7, 14, 28, 56, 112), channels=(64, 128, 256, 512)):
    """(M, N, K) of the im2col GEMM of every 3x3 conv with Cin, Cout in channels."""
    shapes = []
    for h in spatial:
        for cin in channels:
            for cout in channels:
                shapes.append((batch * h * h, cout, 9 * cin))
    return np.array(shapes, dtype=np.int64)


def random_shapes(count=2000, lo=64, hi=8192, seed=5):
    return loguniform_dims(count, lo, hi, seed)
