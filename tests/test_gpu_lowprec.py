"""GPU parity of the per-tile-scaled bf16 / e4m3 gemm and of the quantiser.

Forms (project additions, readings in oracle/precision.py): one float32 scale
per 128 x 128 tile of A and of B; C = alpha * sum_kb sA sB (qA . qB) + beta*C.
Bars: quantiser codes and scales bit-exact against the oracle quantiser;
gemm bit-exact on integer codes with power-of-two scales; against the FP64
product of the dequantised inputs (the kernel-only check), every element
within the bound of tests/scaled_bound.py (float32 accumulation with the
running-sum rescale at each 128-wide K block, plus, for e4m3, the matrix
instruction's alignment of each group of 64 products to the largest) and,
for bf16, normwise <= 1e-5; against the unquantised inputs normwise <= 2e-2
(bf16) / 6e-2 (fp8).
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import precision as P
from paper_1804_10694_amd import inputs
from scaled_bound import scaled_error_bound

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
TOL_UNQUANT = {"bf16": 2e-2, "fp8": 6e-2}
# Normwise kernel-only bar for bf16 (products exact in float32, float32 sums: ~1e-7).
# e4m3 is held to the element-wise bound instead (see scaled_bound.py for the reading of
# v_mfma_scale_f32_32x32x64_f8f6f4 it rests on).
TOL_DEQUANT_BF16 = 1e-5


def _check_dequantised(got, deq, QA, SA, QB, SB, dtype, rows=None, what=""):
    """Element-wise bound (both dtypes) and, for bf16, the normwise bar."""
    bound = scaled_error_bound(QA, SA, QB, SB, dtype, rows=rows)
    err = np.abs(got.astype(np.float64) - deq)
    worst = float(np.max(err / np.maximum(bound, 1e-300)))
    e_deq = oracle.normwise_error(got, deq)
    print(f"{dtype} {what}: vs dequantised normwise {e_deq:.3e}, worst error / bound {worst:.3f}",
          flush=True)
    assert np.all(err <= bound), f"{np.sum(err > bound)} elements past the bound (worst {worst:.3f})"
    if dtype == "bf16":
        assert e_deq <= TOL_DEQUANT_BF16
    return e_deq
CODE_DT = {"bf16": torch.int16, "fp8": torch.uint8}


@pytest.fixture(scope="module")
def tg():
    from paper_1804_10694_amd import tgemm
    tgemm.set_policy("default")
    return tgemm


def _oracle_quant(X, dtype):
    X = np.asarray(X, dtype=np.float32)
    return P.quantize_tiles_e4m3(X) if dtype == "fp8" else P.quantize_tiles_bf16(X)


def _to_dev_codes(Q, dtype):
    if dtype == "bf16":
        return torch.from_numpy(Q.view(np.int16).copy()).to(DEV)
    return torch.from_numpy(Q.copy()).to(DEV)


def _gemm_scaled(tg, QA, SA, QB, SB, C0, alpha, beta, dtype, sid=None, pad=0):
    """GPU C = alpha * dequant product + beta*C0 from oracle-made codes and scales."""
    qa, qb = _to_dev_codes(QA, dtype), _to_dev_codes(QB, dtype)
    if pad:
        qa = torch.nn.functional.pad(qa, (0, pad))[:, :QA.shape[1]]
        qb = torch.nn.functional.pad(qb, (0, pad))[:, :QB.shape[1]]
    sa = torch.from_numpy(SA).to(DEV)
    sb = torch.from_numpy(SB).to(DEV)
    C = torch.as_tensor(C0, dtype=torch.float32).clone().to(DEV)
    if sid is None:
        tg.gemm_scaled(qa, sa, qb, sb, C, alpha, beta, dtype)
    else:
        # schedule pinned: scales of exactly 1 let the unscaled entry point run it
        assert np.all(SA == 1) and np.all(SB == 1)
        tg.gemm_with_schedule(qa, qb, C, alpha, beta, dtype, sid)
    torch.cuda.synchronize()
    return C.cpu().numpy()


# ------------------------------------------------------------------ quantiser
@pytest.mark.parametrize("dtype", ["fp8", "bf16"])
@pytest.mark.parametrize("shape", [(300, 260), (128, 128), (1, 5), (129, 1000)])
def test_quantiser_bit_exact(tg, dtype, shape):
    A, _ = inputs.lowprec_inputs(shape[0], 4, shape[1], seed=31)
    Qr, Sr = _oracle_quant(A.numpy(), dtype)
    Q, S = tg.quantize_tiles(A.to(DEV), dtype)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(S.cpu().numpy(), Sr)
    Qg = Q.cpu().numpy()
    if dtype == "bf16":
        Qg = Qg.view(np.uint16)
    np.testing.assert_array_equal(Qg, Qr)


@pytest.mark.parametrize("dtype", ["fp8", "bf16"])
@pytest.mark.parametrize("pad", [0, 3], ids=["aligned", "ld+3"])
def test_quantiser_full_tiles_both_load_widths(tg, dtype, pad):
    # whole 128 x 128 tiles: aligned rows take the 16-byte loads, a row stride of
    # cols + 3 the per-element ones; a ragged last row and column of tiles too
    rows, cols = 300, 388
    A, _ = inputs.lowprec_inputs(rows, 4, cols, seed=33)
    Xw = torch.full((rows, cols + pad), float("nan"))
    Xw[:, :cols] = A
    Xd = Xw.to(DEV)[:, :cols]
    Qr, Sr = _oracle_quant(A.numpy(), dtype)
    Q, S = tg.quantize_tiles(Xd, dtype)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(S.cpu().numpy(), Sr)
    Qg = Q.cpu().numpy()
    if dtype == "bf16":
        Qg = Qg.view(np.uint16)
    np.testing.assert_array_equal(Qg, Qr)


def test_quantiser_special_values(tg):
    # ties, saturation, subnormal codes and signed zero inside one tile
    vals = np.array([448.0, -448.0, 1.0625, 1.1875, 0.0009765625, 0.0029296875, -0.0, 0.0,
                     3.0e-3, 7.5, -240.0, 17.0], dtype=np.float32)
    X = np.zeros((4, 16), dtype=np.float32)
    X[0, :len(vals)] = vals
    Qr, Sr = P.quantize_tiles_e4m3(X)
    assert Sr[0, 0] == 1.0
    Q, S = tg.quantize_tiles(torch.from_numpy(X).to(DEV), "fp8")
    np.testing.assert_array_equal(Q.cpu().numpy(), Qr)


# ------------------------------------------------------------------ gemm exact
@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_every_schedule_bit_exact_integer_codes(tg, dtype):
    # Integer values up to 16 are exact codes in both formats (scale 1).  Ragged shapes
    # exercise partial tiles and the K remainder; vec=1 schedules also get padded strides.
    M, N, K = 300, 208, 272   # row strides of 16-byte multiples for the vec=4 schedules
    A, B, C0 = inputs.integer_inputs(M, N, K, seed=32, r=16)
    ones_a = np.ones(P.scale_grid_shape(M, K), np.float32)
    ones_b = np.ones(P.scale_grid_shape(K, N), np.float32)
    if dtype == "fp8":
        QA, QB = P.e4m3_encode(A.numpy().astype(np.float64)), P.e4m3_encode(B.numpy().astype(np.float64))
    else:
        QA, QB = P.bf16_bits(A.numpy()), P.bf16_bits(B.numpy())
    ref = oracle.gemm(A, B, C0, 1.5, 0.5)
    for sid, info in tg.schedules(dtype):
        pad = 0 if info["vec"] == 4 else 3
        got = _gemm_scaled(tg, QA, ones_a, QB, ones_b, C0.numpy(), 1.5, 0.5, dtype, sid=sid, pad=pad)
        np.testing.assert_array_equal(got.astype(np.float64), ref, err_msg=f"schedule {sid} {info}")
    # the scaled entry point with unit scales gives the same bits
    got = _gemm_scaled(tg, QA, ones_a, QB, ones_b, C0.numpy(), 1.5, 0.5, dtype)
    np.testing.assert_array_equal(got.astype(np.float64), ref)


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_power_of_two_scales_exact(tg, dtype):
    # integer codes with scales in {1/2, 1, 2, 4}: every partial sum and every scaled
    # fold is exact, so the result equals the oracle bit for bit
    M, N, K = 260, 300, 384
    A, B, _ = inputs.integer_inputs(M, N, K, seed=33, r=8)
    g = np.random.default_rng(34)
    SA = (2.0 ** g.integers(-1, 3, P.scale_grid_shape(M, K))).astype(np.float32)
    SB = (2.0 ** g.integers(-1, 3, P.scale_grid_shape(K, N))).astype(np.float32)
    if dtype == "fp8":
        QA, QB = P.e4m3_encode(A.numpy().astype(np.float64)), P.e4m3_encode(B.numpy().astype(np.float64))
    else:
        QA, QB = P.bf16_bits(A.numpy()), P.bf16_bits(B.numpy())
    ref = P.gemm_scaled_expected(QA, SA, QB, SB, None, 1.0, 0.0, dtype)
    got = _gemm_scaled(tg, QA, SA, QB, SB, np.full((M, N), np.nan, np.float32), 1.0, 0.0, dtype)
    np.testing.assert_array_equal(got.astype(np.float64), ref)


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_packed_schedules_scaled_exact(tg, dtype):
    # Every packed schedule (operands copied, B transposed, zero-padded) through the scaled
    # entry point: integer codes with power-of-two scales that change across K blocks, so
    # the running-sum rescaling at every 128-wide K block is exercised and must be exact.
    M, N, K = 300, 270, 520
    A, B, _ = inputs.integer_inputs(M, N, K, seed=37, r=8)
    g = np.random.default_rng(38)
    SA = (2.0 ** g.integers(-2, 3, P.scale_grid_shape(M, K))).astype(np.float32)
    SB = (2.0 ** g.integers(-2, 3, P.scale_grid_shape(K, N))).astype(np.float32)
    if dtype == "fp8":
        QA, QB = P.e4m3_encode(A.numpy().astype(np.float64)), P.e4m3_encode(B.numpy().astype(np.float64))
    else:
        QA, QB = P.bf16_bits(A.numpy()), P.bf16_bits(B.numpy())
    C0 = np.random.default_rng(39).integers(-4, 5, (M, N)).astype(np.float32)
    ref = P.gemm_scaled_expected(QA, SA, QB, SB, C0, 1.0, 0.5, dtype)
    packed = [sid for sid, info in tg.schedules(dtype) if info["vec"] == 0]
    assert packed
    try:
        for sid in packed:
            tg.set_policy(f"force:{sid}")
            got = _gemm_scaled(tg, QA, SA, QB, SB, C0, 1.0, 0.5, dtype)
            np.testing.assert_array_equal(got.astype(np.float64), ref, err_msg=f"schedule {sid}")
    finally:
        tg.set_policy("default")


@pytest.mark.parametrize("dtype,K", [("bf16", 2048), ("fp8", 4096)])
def test_packed_schedules_scaled_exact_padded_row_pitch(tg, dtype, K):
    # K * element size a multiple of 4 KB: the packed rows get 512 bytes of padding past K;
    # integer codes, power-of-two scales changing across K blocks, every packed schedule exact
    M, N = 300, 270
    A, B, _ = inputs.integer_inputs(M, N, K, seed=41 + K, r=8)
    g = np.random.default_rng(42)
    SA = (2.0 ** g.integers(-2, 3, P.scale_grid_shape(M, K))).astype(np.float32)
    SB = (2.0 ** g.integers(-2, 3, P.scale_grid_shape(K, N))).astype(np.float32)
    if dtype == "fp8":
        QA, QB = P.e4m3_encode(A.numpy().astype(np.float64)), P.e4m3_encode(B.numpy().astype(np.float64))
    else:
        QA, QB = P.bf16_bits(A.numpy()), P.bf16_bits(B.numpy())
    C0 = np.random.default_rng(43).integers(-4, 5, (M, N)).astype(np.float32)
    ref = P.gemm_scaled_expected(QA, SA, QB, SB, C0, 1.0, 0.5, dtype)
    packed = [sid for sid, info in tg.schedules(dtype) if info["vec"] == 0]
    assert packed
    try:
        for sid in packed:
            print(f"packed schedule {sid} {dtype} K={K}", flush=True)
            tg.set_policy(f"force:{sid}")
            got = _gemm_scaled(tg, QA, SA, QB, SB, C0, 1.0, 0.5, dtype)
            np.testing.assert_array_equal(got.astype(np.float64), ref, err_msg=f"schedule {sid}")
    finally:
        tg.set_policy("default")


# ------------------------------------------------------------------ tolerance
@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
@pytest.mark.parametrize("shape", [(512, 512, 1024), (300, 389, 517)])
def test_lowprec_tolerances(tg, dtype, shape):
    M, N, K = shape
    A, B = inputs.lowprec_inputs(M, N, K, seed=30)
    QA, SA = _oracle_quant(A.numpy(), dtype)
    QB, SB = _oracle_quant(B.numpy(), dtype)
    C0 = np.zeros((M, N), np.float32)
    got = _gemm_scaled(tg, QA, SA, QB, SB, C0, 1.0, 0.0, dtype)
    deq = P.gemm_scaled_expected(QA, SA, QB, SB, None, 1.0, 0.0, dtype)
    unq = oracle.gemm(A, B, None, 1.0, 0.0)
    _check_dequantised(got, deq, QA, SA, QB, SB, dtype, what=str(shape))
    e_unq = oracle.normwise_error(got, unq)
    print(f"{dtype} {shape}: vs unquantised {e_unq:.3e}")
    assert e_unq <= TOL_UNQUANT[dtype]


def _spread_codes(rows, cols, rng, dtype):
    """Values whose exponents spread over about 14 binades, on the dtype's grid."""
    mag = 2.0 ** rng.uniform(-7, 7.5, (rows, cols)) * rng.choice([-1.0, 1.0], (rows, cols))
    if dtype == "fp8":
        return P.e4m3_encode(P.e4m3_rne_sat(mag))
    return P.bf16_bits(P.bf16_rne(mag.astype(np.float32)))


@pytest.mark.parametrize("dtype", ["fp8", "bf16"])
@pytest.mark.parametrize("shape", [(256, 320, 1024), (200, 136, 2100)])
def test_elementwise_bound_wide_exponent_spread(tg, dtype, shape):
    # Codes spread over ~14 binades (products over ~28) and scale products that are not
    # powers of two: the inputs on which the e4m3 instruction's alignment and the running
    # sum's rescale at each K block lose the most.  Every element within the bound.
    M, N, K = shape
    rng = np.random.default_rng(64 + K)
    QA, QB = _spread_codes(M, K, rng, dtype), _spread_codes(K, N, rng, dtype)
    SA = rng.uniform(0.3, 3.0, P.scale_grid_shape(M, K)).astype(np.float32)
    SB = rng.uniform(0.3, 3.0, P.scale_grid_shape(K, N)).astype(np.float32)
    got = _gemm_scaled(tg, QA, SA, QB, SB, np.zeros((M, N), np.float32), 1.0, 0.0, dtype)
    deq = P.gemm_scaled_expected(QA, SA, QB, SB, None, 1.0, 0.0, dtype)
    _check_dequantised(got, deq, QA, SA, QB, SB, dtype, what=f"spread {shape}")


def test_fp8_mfma_exact_within_one_binade(tg):
    # Products that share a binade are summed exactly by the e4m3 MFMA, so the kernel's
    # own arithmetic (packing, k pairing, scale folds) must reproduce the FP64 result
    # bit for bit on such inputs with non-trivial mantissas.
    rng = np.random.default_rng(36)
    M, N, K = 256, 192, 384
    A = P.e4m3_rne_sat(rng.uniform(1, 2, (M, K)) * rng.choice([-1, 1], (M, K)))
    B = P.e4m3_rne_sat(rng.uniform(1, 2, (K, N)) * rng.choice([-1, 1], (K, N)))
    QA, QB = P.e4m3_encode(A), P.e4m3_encode(B)
    SA = np.ones(P.scale_grid_shape(M, K), np.float32)
    SB = np.ones(P.scale_grid_shape(K, N), np.float32)
    ref = P.gemm_scaled_expected(QA, SA, QB, SB, None, 1.0, 0.0, "fp8")
    got = _gemm_scaled(tg, QA, SA, QB, SB, np.zeros((M, N), np.float32), 1.0, 0.0, "fp8")
    np.testing.assert_array_equal(got.astype(np.float64), ref)


def test_scaled_validation(tg):
    f = 0x10000
    lib = tg.lib
    # scale pointers are required when A and B are read
    assert lib.tgemm_scaled(4, 4, 4, 1.0, f, 4, None, f, 4, f, 0.0, f, 4, 3, None) == 1
    assert lib.tgemm_scaled(4, 4, 4, 1.0, f, 4, f, f, 4, None, 0.0, f, 4, 2, None) == 1
    # float32 dtypes are not scaled forms
    assert lib.tgemm_scaled(4, 4, 4, 1.0, f, 4, f, f, 4, f, 0.0, f, 4, 0, None) == 2
    assert lib.tgemm_quantize_tiles(4, 4, f, 3, f, 4, f, 3, None) == 1   # ldx < cols
    assert lib.tgemm_quantize_tiles(4, 4, f, 4, f, 4, f, 1, None) == 2   # x3 is not a code type


# ------------------------------------------------------------------ full size, sampled
@pytest.mark.parametrize("dtype", ["fp8", "bf16"])
def test_full_size_16384_sampled(tg, dtype):
    # 16384^3: A, B ~ N(0,1) with 1% of rows x1e3 (seed 30); quantised by the oracle on
    # the CPU; the GPU quantiser must give the same codes; sampled rows of C are checked.
    M = N = K = 16384
    A, B = inputs.lowprec_inputs(M, N, K, seed=30)
    QB, SB = _oracle_quant(B.numpy(), dtype)
    rng = np.random.default_rng(35)
    rows = np.sort(rng.choice(M, size=6, replace=False))
    tiles = sorted(set((rows // 128).tolist()))
    # the A row-tiles holding the sampled rows, quantised by the oracle
    A_np = A.numpy()
    QA = np.zeros((M, K), dtype=np.uint8 if dtype == "fp8" else np.uint16)
    SA = np.ones(P.scale_grid_shape(M, K), np.float32)
    for ti in tiles:
        q, s = _oracle_quant(A_np[ti * 128:(ti + 1) * 128], dtype)
        QA[ti * 128:(ti + 1) * 128] = q
        SA[ti] = s[0]
    # GPU quantiser on the full matrices; its B codes must match the oracle's
    Qa_dev, Sa_dev = tg.quantize_tiles(A.to(DEV), dtype)
    Qb_dev, Sb_dev = tg.quantize_tiles(B.to(DEV), dtype)
    qb_ref = _to_dev_codes(QB, dtype)
    assert torch.equal(Qb_dev.view(qb_ref.dtype), qb_ref)
    assert torch.equal(Sb_dev.cpu(), torch.from_numpy(SB))
    for ti in tiles:
        sl = slice(ti * 128, (ti + 1) * 128)
        assert torch.equal(Qa_dev[sl].view(qb_ref.dtype), _to_dev_codes(QA[sl], dtype))
        assert torch.equal(Sa_dev[ti].cpu(), torch.from_numpy(SA[ti]))
    C = torch.zeros(M, N, device=DEV)
    tg.gemm_scaled(Qa_dev, Sa_dev, Qb_dev, Sb_dev, C, 1.0, 0.0, dtype)
    torch.cuda.synchronize()
    got = C[torch.from_numpy(rows).to(DEV)].cpu().numpy()
    # dequantised rows of A (their own row tiles) and all of B, in FP64
    Arows = np.stack([P.decode(QA[r], dtype) for r in rows])
    for n, r in enumerate(rows):
        Arows[n] *= np.repeat(SA[r // 128].astype(np.float64), 128)[:K]
    Bd = P.dequantize_tiles(P.decode(QB, dtype), SB, 128)
    deq = oracle.gemm(Arows, Bd, None, 1.0, 0.0)
    unq = oracle.gemm_rows(A, B, None, 1.0, 0.0, rows)
    _check_dequantised(got, deq, QA, SA, QB, SB, dtype, rows=rows, what="16384^3 sampled rows")
    e_unq = oracle.normwise_error(got, unq)
    print(f"{dtype} 16384^3 sampled rows: vs unquantised {e_unq:.3e}")
    assert e_unq <= TOL_UNQUANT[dtype]
