"""CPU checks of the element-wise error bound used by the scaled-gemm GPU tests
(tests/scaled_bound.py): the bound holds for a float32 emulation of the kernel's
arithmetic under the stated reading of the e4m3 matrix instruction, on inputs
chosen to make that reading matter (products spread over many binades, scale
products that are not powers of two), and it is not vacuous: an emulated
instruction that keeps half as many bits exceeds it.
"""
import numpy as np
import pytest

from oracle import precision as P
from scaled_bound import emulate_scaled_gemm, scaled_error_bound


def _spread_codes(rows, cols, rng, dtype):
    """Values whose exponents spread over about 14 binades, on the dtype's grid."""
    mag = 2.0 ** rng.uniform(-7, 7.5, (rows, cols)) * rng.choice([-1.0, 1.0], (rows, cols))
    if dtype == "fp8":
        return P.e4m3_encode(P.e4m3_rne_sat(mag))
    return P.bf16_bits(P.bf16_rne(mag.astype(np.float32)))


def _scales(shape, rng):
    return rng.uniform(0.3, 3.0, shape).astype(np.float32)


@pytest.mark.parametrize("dtype", ["fp8", "bf16"])
def test_bound_holds_for_the_emulated_kernel(dtype):
    rng = np.random.default_rng(61)
    M, N, K = 5, 7, 300          # three K blocks, the last one partial
    QA, QB = _spread_codes(M, K, rng, dtype), _spread_codes(K, N, rng, dtype)
    SA = _scales(P.scale_grid_shape(M, K), rng)
    SB = _scales(P.scale_grid_shape(K, N), rng)
    deq = P.gemm_scaled_expected(QA, SA, QB, SB, None, 1.0, 0.0, dtype)
    emu = emulate_scaled_gemm(QA, SA, QB, SB, dtype).astype(np.float64)
    bound = scaled_error_bound(QA, SA, QB, SB, dtype)
    err = np.abs(emu - deq)
    assert np.all(err <= bound), np.max(err / bound)
    # the error is real (not zero) for fp8, where the truncation is the larger part
    if dtype == "fp8":
        assert np.max(err) > 0


def test_bound_is_not_vacuous():
    # emulating an instruction that keeps only 7 bits must break the 14-bit bound (on
    # these inputs the emulated 14-bit error stays about 26 times below the bound, and
    # 8 kept bits already exceed it)
    rng = np.random.default_rng(62)
    M, N, K = 6, 6, 256
    QA, QB = _spread_codes(M, K, rng, "fp8"), _spread_codes(K, N, rng, "fp8")
    SA = _scales(P.scale_grid_shape(M, K), rng)
    SB = _scales(P.scale_grid_shape(K, N), rng)
    deq = P.gemm_scaled_expected(QA, SA, QB, SB, None, 1.0, 0.0, "fp8")
    emu7 = emulate_scaled_gemm(QA, SA, QB, SB, "fp8", kept_bits=7).astype(np.float64)
    bound14 = scaled_error_bound(QA, SA, QB, SB, "fp8", kept_bits=14)
    assert np.any(np.abs(emu7 - deq) > bound14)


def test_emulation_is_exact_within_one_binade():
    # products in one binade lose nothing to the alignment: the emulation equals the
    # float32 rounding of a float32 running sum, which on integers is exact
    rng = np.random.default_rng(63)
    A = rng.integers(-8, 9, (4, 256)).astype(np.float64)
    B = rng.integers(-8, 9, (256, 4)).astype(np.float64)
    QA, QB = P.e4m3_encode(A), P.e4m3_encode(B)
    ones_a = np.ones(P.scale_grid_shape(4, 256), np.float32)
    ones_b = np.ones(P.scale_grid_shape(256, 4), np.float32)
    emu = emulate_scaled_gemm(QA, ones_a, QB, ones_b, "fp8")
    np.testing.assert_array_equal(emu.astype(np.float64), A @ B)
