"""GPU parity of the cost model's network kernels against the FP64 oracle (oracle/mlp.py).

Forward, loss and chain-rule gradients run on the library's own F32 gemm plus
element-wise kernels; bars: normwise relative error <= 1e-4 for outputs and
gradients (FP32 against FP64), <= 1e-6 relative for the Adam update on
identical inputs.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import mlp as O

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
DIMS = [20, 256, 256, 256, 1]


@pytest.fixture(scope="module")
def tg():
    from paper_1804_10694_amd import tgemm
    return tgemm


def _init(dims, seed):
    """He-normal weights, small biases, float32."""
    r = np.random.default_rng(seed)
    parts = []
    for l in range(len(dims) - 1):
        parts.append(r.standard_normal(dims[l] * dims[l + 1]) * np.sqrt(2.0 / dims[l]))
        parts.append(r.standard_normal(dims[l + 1]) * 0.1)
    return np.concatenate(parts).astype(np.float32)


def _data(rows, seed, f=20):
    r = np.random.default_rng(seed)
    X = r.standard_normal((rows, f)).astype(np.float32)
    y = (np.sin(X[:, 0]) + 0.5 * X[:, 1] * X[:, 2] - 0.2 * X[:, 3]).astype(np.float32)
    return X, y


@pytest.mark.parametrize("rows", [1, 37, 300, 1024])
def test_forward_matches_oracle(tg, rows):
    p = _init(DIMS, 1)
    assert tg.mlp_param_count(DIMS) == len(p) == O.param_count(DIMS)
    X, _ = _data(rows, 2)
    out = tg.mlp_forward(DIMS, torch.from_numpy(p).to(DEV), torch.from_numpy(X).to(DEV))
    torch.cuda.synchronize()
    ref, _ = O.forward(p.astype(np.float64), DIMS, X.astype(np.float64))
    assert oracle.normwise_error(out.cpu().numpy(), ref) <= 1e-4


@pytest.mark.parametrize("dims,rows", [(DIMS, 300), ([7, 33, 1], 65), ([20, 64, 64, 64, 1], 512)])
def test_gradients_and_loss_match_oracle(tg, dims, rows):
    p = _init(dims, 3)
    X, y = _data(rows, 4, f=dims[0])
    P = torch.from_numpy(p).to(DEV)
    G = torch.zeros_like(P)
    m, v = torch.zeros_like(P), torch.zeros_like(P)
    loss = torch.zeros(1, device=DEV)
    work = tg.mlp_workspace(dims, rows)
    tg.mlp_train_step(dims, P, G, m, v, 1, 0.0, torch.from_numpy(X).to(DEV),
                      torch.from_numpy(y).to(DEV), loss, work)
    torch.cuda.synchronize()
    L, g = O.gradients(p.astype(np.float64), dims, X.astype(np.float64), y.astype(np.float64))
    assert abs(loss.item() - L) <= 1e-5 * abs(L)
    assert oracle.normwise_error(G.cpu().numpy(), g) <= 1e-4
    # per layer too, so that a small layer cannot hide behind a large one
    off = 0
    for l in range(len(dims) - 1):
        n = dims[l] * dims[l + 1] + dims[l + 1]
        assert oracle.normwise_error(G.cpu().numpy()[off:off + n], g[off:off + n]) <= 1e-4, l
        off += n
    assert torch.equal(P.cpu(), torch.from_numpy(p))      # lr = 0 leaves the parameters


@pytest.mark.parametrize("step", [1, 2, 17, 1000])
def test_adam_step_matches_oracle(tg, step):
    r = np.random.default_rng(5 + step)
    n = 5000
    p = r.standard_normal(n).astype(np.float32)
    g = (r.standard_normal(n) * 10.0 ** r.integers(-6, 1, n)).astype(np.float32)
    m = (r.standard_normal(n) * 0.01).astype(np.float32)
    v = (r.random(n) * 1e-3).astype(np.float32)
    P, Gd, Md, Vd = (torch.from_numpy(a.copy()).to(DEV) for a in (p, g, m, v))
    tg.adam_step(P, Gd, Md, Vd, step, 1e-3)
    torch.cuda.synchronize()
    p2, m2, v2 = O.adam_step(p, g, m, v, step, 1e-3)
    upd_ref = p2 - p.astype(np.float64)
    upd = P.cpu().numpy().astype(np.float64) - p.astype(np.float64)
    # the float32 parameter store rounds the update: compare against 1e-6 of the
    # update plus the rounding of the stored value
    tol = 1e-6 * np.abs(upd_ref) + np.abs(p) * 2.0 ** -23
    assert np.all(np.abs(upd - upd_ref) <= tol)
    assert oracle.normwise_error(Md.cpu().numpy(), m2) <= 1e-6
    assert oracle.normwise_error(Vd.cpu().numpy(), v2) <= 1e-6


def test_training_loss_falls(tg):
    dims = DIMS
    X, y = _data(2048, 6)
    P = torch.from_numpy(_init(dims, 7)).to(DEV)
    G, m, v = torch.zeros_like(P), torch.zeros_like(P), torch.zeros_like(P)
    loss = torch.zeros(1, device=DEV)
    Xd, yd = torch.from_numpy(X).to(DEV), torch.from_numpy(y).to(DEV)
    batch = 256
    work = tg.mlp_workspace(dims, batch)
    losses = []
    step = 0
    for epoch in range(30):
        for b0 in range(0, 2048, batch):
            step += 1
            tg.mlp_train_step(dims, P, G, m, v, step, 1e-3, Xd[b0:b0 + batch], yd[b0:b0 + batch],
                              loss, work)
        torch.cuda.synchronize()
        losses.append(O.loss(P.cpu().numpy().astype(np.float64), dims, X, y))
    print("loss by epoch:", [round(x, 4) for x in losses[::5]])
    assert losses[-1] < 0.1 * losses[0]


def test_mlp_validation(tg):
    d = (tg.ctypes.c_int32 * 3)(4, 8, 2)   # last width must be 1
    assert tg.lib.tgemm_mlp_param_count(2, d) == -1
    d = (tg.ctypes.c_int32 * 3)(4, 8, 1)
    assert tg.lib.tgemm_mlp_param_count(2, d) == 4 * 8 + 8 + 8 + 1
    assert tg.lib.tgemm_mlp_workspace_count(2, d, 0) == -1
