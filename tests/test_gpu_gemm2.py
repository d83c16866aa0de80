"""GPU parity of the back-to-back gemm (tgemm_gemm2) against the FP64 oracle.

Operation: E = alpha * act(A B) D + beta * E, act = identity or ReLU, with act(A B) kept on
chip (the fused layer pair of the Tiramisu paper's VGG block, Section VI-A).  Bars as for the
gemm: bit-exact on small-integer inputs (every partial sum of both products an integer below
2^24, each intermediate value exactly the sum of its bf16 high and low parts), normwise
relative error <= 1e-5 for f32 and x3 on U[-1, 1] inputs.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import gemm2 as OG
from paper_1804_10694_amd import inputs

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def tg():
    from paper_1804_10694_amd import tgemm
    return tgemm


def _inputs(M, K, N1, N2, seed, integer):
    g = torch.Generator().manual_seed(seed)
    if integer:
        mk = lambda r, c: torch.randint(-4, 5, (r, c), generator=g).float()   # noqa: E731
    else:
        mk = lambda r, c: 2 * torch.rand(r, c, generator=g) - 1                # noqa: E731
    return mk(M, K), mk(K, N1), mk(N1, N2), mk(M, N2)


def _run(tg, A, B, D, E0, alpha, beta, relu, dtype):
    E = E0.clone().to(DEV)
    tg.gemm2(A.to(DEV), B.to(DEV), D.to(DEV), E, alpha, beta, relu, dtype)
    torch.cuda.synchronize()
    return E.cpu()


# (M, K, N1, N2): one element; whole 64-row blocks; ragged everything (4-byte loads); N1 in
# (128, 256] (the wide kernel) with several 256-column chunks of E; deep K; K = 1
SHAPES = [(1, 4, 4, 4), (64, 16, 64, 64), (65, 17, 33, 300), (130, 64, 128, 256), (200, 100, 256, 520),
          (3, 300, 250, 7), (129, 1, 129, 129), (64, 48, 200, 64)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("relu", [False, True], ids=["id", "relu"])
@pytest.mark.parametrize("dtype", ["f32", "x3"])
def test_integer_inputs_bit_exact(tg, dtype, relu, shape):
    print(f"gemm2 {dtype} relu={relu} {shape}", flush=True)
    A, B, D, E0 = _inputs(*shape, seed=sum(shape), integer=True)
    ref = OG.gemm2(A, B, D, E0, 1.5, 0.5, relu)
    got = _run(tg, A, B, D, E0, 1.5, 0.5, relu, dtype)
    np.testing.assert_array_equal(got.numpy().astype(np.float64), ref, err_msg=f"{dtype} {shape}")


@pytest.mark.parametrize("dtype", ["f32", "x3"])
def test_nan_padded_strides(tg, dtype):
    # A, B, D inside buffers with NaN columns past the matrices (aligned and unaligned pads):
    # nothing past K or N1 may reach E, and E's canary columns stay NaN
    for p, (M, K, N1, N2) in enumerate([(70, 36, 100, 130), (64, 33, 17, 260)]):
        A, B, D, E0 = _inputs(M, K, N1, N2, seed=90 + p, integer=True)
        pad = 4 if p == 0 else 3
        Ab, Bb, Db, Eb = (inputs.padded(x, pad)[0].to(DEV) for x in (A, B, D, E0))
        Ad, Bd, Dd, Ed = Ab[:, :K], Bb[:, :N1], Db[:, :N2], Eb[:, :N2]
        tg.gemm2(Ad, Bd, Dd, Ed, 1.0, 1.0, True, dtype)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(Ed.cpu().numpy().astype(np.float64), OG.gemm2(A, B, D, E0, 1.0, 1.0, True))
        assert torch.isnan(Eb[:, N2:]).all()


@pytest.mark.parametrize("shape", [(1000, 256, 256, 256), (333, 77, 130, 90)])
@pytest.mark.parametrize("relu", [False, True], ids=["id", "relu"])
@pytest.mark.parametrize("dtype", ["f32", "x3"])
def test_uniform_inputs_within_tolerance(tg, dtype, relu, shape):
    A, B, D, E0 = _inputs(*shape, seed=7 + sum(shape), integer=False)
    ref = OG.gemm2(A, B, D, E0, 1.0, 1.0, relu)
    err = oracle.normwise_error(_run(tg, A, B, D, E0, 1.0, 1.0, relu, dtype).numpy(), ref)
    print(f"{dtype} relu={relu} {shape} normwise error {err:.3e}")
    assert err <= 1e-5


def test_same_result_as_two_gemm_calls(tg):
    # integer inputs: the fused kernel and two library gemms with the ReLU between agree bit for bit
    A, B, D, E0 = _inputs(300, 64, 192, 100, seed=95, integer=True)
    Ad, Bd, Dd = A.to(DEV), B.to(DEV), D.to(DEV)
    T = torch.zeros(300, 192, device=DEV)
    tg.gemm(Ad, Bd, T, 1.0, 0.0, "f32")
    torch.relu_(T)
    E2 = E0.clone().to(DEV)
    tg.gemm(T, Dd, E2, 2.0, -1.0, "f32")
    got = _run(tg, A, B, D, E0, 2.0, -1.0, True, "f32")
    assert torch.equal(got, E2.cpu())


def test_degenerate_cases(tg):
    A, B, D, E0 = _inputs(70, 12, 20, 30, seed=96, integer=True)
    # alpha == 0 and K == 0: E = beta * E, A, B, D not read (NaN there)
    nan = torch.full_like(A, float("nan"))
    np.testing.assert_array_equal(_run(tg, nan, B, D, E0, 0.0, 0.5, True, "f32").numpy(), (0.5 * E0).numpy())
    Ez = E0.clone().to(DEV)
    tg.gemm2(torch.zeros(70, 0, device=DEV), torch.zeros(0, 20, device=DEV), D.to(DEV), Ez, 1.0, 2.0)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(Ez.cpu().numpy(), (2.0 * E0).numpy())
    # beta == 0 does not read E (NaN there)
    got = _run(tg, A, B, D, torch.full_like(E0, float("nan")), 1.0, 0.0, False, "x3")
    np.testing.assert_array_equal(got.numpy().astype(np.float64), OG.gemm2(A, B, D))
    # N1 above 256 is refused; an unknown activation too
    with pytest.raises(tg.TgemmError):
        tg.gemm2(A.to(DEV), torch.zeros(12, 257, device=DEV), torch.zeros(257, 30, device=DEV), E0.to(DEV))
    Ad = A.to(DEV)
    rc = tg.lib.tgemm_gemm2(70, 20, 30, 12, 1.0, Ad.data_ptr(), 12, Ad.data_ptr(), 20, 7, Ad.data_ptr(), 30,
                            0.0, Ad.data_ptr(), 30, 0, None)
    assert rc == tg.INVALID_VALUE


@pytest.mark.parametrize("dtype", ["f32", "x3"])
def test_full_size_sampled_rows(tg, dtype):
    # the benchmark's pair of 256-wide layers over 32 x 56 x 56 pixels, sampled rows vs the oracle
    M, K, N1, N2 = 32 * 56 * 56, 256, 256, 256
    A, B, D, E0 = _inputs(M, K, N1, N2, seed=97, integer=False)
    got = _run(tg, A, B, D, E0, 1.0, 1.0, True, dtype)
    rows = np.concatenate([np.random.default_rng(98).choice(M, 300, replace=False), [0, 63, 64, M - 1]])
    ref = OG.gemm2(A, B, D, E0, 1.0, 1.0, True, rows=rows)
    err = oracle.normwise_error(got[torch.from_numpy(rows)].numpy(), ref)
    print(f"{dtype} full-size sampled normwise error {err:.3e}")
    assert err <= 1e-5
