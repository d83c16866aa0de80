"""Pins of the oracle against facts fixed outside it (no GPU needed).

gemm: the problem statement of the Tiramisu paper, Section I
(C = alpha*A*B + beta*C).  Precision forms: bfloat16 and OCP E4M3FN rounding
definitions (golden files cite them) and closed forms of the split product.
"""
import os

import numpy as np
import pytest
import torch

import oracle
from oracle import precision as P
from paper_1804_10694_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(seed):
    return np.random.default_rng(seed)


# ----------------------------------------------------------------- gemm
@pytest.mark.parametrize("M,N,K", [(64, 64, 64), (97, 131, 53), (300, 17, 512), (1, 1, 1),
                                   (5, 300, 2)])
def test_gemm_matches_numpy_float64(M, N, K):
    r = _rng(M * 7 + N * 3 + K)
    A, B, C0 = r.standard_normal((M, K)), r.standard_normal((K, N)), r.standard_normal((M, N))
    ref = 1.5 * (A @ B) + 0.5 * C0          # library matmul, independent of the oracle
    got = oracle.gemm(A, B, C0, 1.5, 0.5)
    assert oracle.normwise_error(got, ref) <= 1e-13


def test_gemm_integer_inputs_exact():
    # Integer products and sums below 2^53 are exact in FP64, so the oracle must equal
    # integer arithmetic bit for bit.  Non-square shapes catch a transposed operand.
    r = _rng(11)
    M, N, K = 37, 53, 71
    A = r.integers(-50, 51, (M, K))
    B = r.integers(-50, 51, (K, N))
    C0 = r.integers(-50, 51, (M, N))
    exact = 3 * (A.astype(object) @ B.astype(object)) - 2 * C0.astype(object)
    got = oracle.gemm(A.astype(np.float64), B.astype(np.float64), C0.astype(np.float64), 3.0, -2.0)
    assert np.array_equal(got, np.array(exact, dtype=np.float64))


def test_gemm_identity_closed_form():
    r = _rng(12)
    K, N = 45, 29
    B, C0 = r.standard_normal((K, N)), r.standard_normal((K, N))
    got = oracle.gemm(np.eye(K), B, C0, 1.25, -0.75)
    assert np.array_equal(got, 1.25 * B + (-0.75) * C0)


def test_gemm_alpha_zero_is_beta_c():
    r = _rng(13)
    A = np.full((8, 9), np.nan)             # alpha == 0: A and B are not read
    B = np.full((9, 7), np.nan)
    C0 = r.standard_normal((8, 7))
    assert np.array_equal(oracle.gemm(A, B, C0, 0.0, 0.5), 0.5 * C0)


def test_gemm_k_zero_is_beta_c():
    C0 = _rng(14).standard_normal((6, 5))
    got = oracle.gemm(np.zeros((6, 0)), np.zeros((0, 5)), C0, 2.0, 3.0)
    assert np.array_equal(got, 3.0 * C0)


def test_gemm_beta_zero_does_not_read_c():
    r = _rng(15)
    A, B = r.standard_normal((10, 12)), r.standard_normal((12, 11))
    C0 = np.full((10, 11), np.nan)
    got = oracle.gemm(A, B, C0, 1.0, 0.0)
    assert not np.isnan(got).any()
    assert oracle.normwise_error(got, A @ B) <= 1e-14


def test_gemm_rank_one_closed_form():
    # A = u v^T, B = w x^T  ->  A B = (v . w) u x^T, exact for small integers.
    r = _rng(16)
    M, K, N = 23, 31, 19
    u, v = r.integers(-9, 10, M), r.integers(-9, 10, K)
    w, x = r.integers(-9, 10, K), r.integers(-9, 10, N)
    A = np.outer(u, v).astype(np.float64)
    B = np.outer(w, x).astype(np.float64)
    expect = float(v @ w) * np.outer(u, x).astype(np.float64)
    assert np.array_equal(oracle.gemm(A, B, None, 1.0, 0.0), expect)


def test_gemm_rows_agree_with_full():
    A, B, C0 = inputs.gemm_inputs(70, 40, 33, 3)
    full = oracle.gemm(A, B, C0, 1.0, 1.0)
    rows = np.array([0, 5, 69, 33])
    part = oracle.gemm_rows(A, B, C0, 1.0, 1.0, rows)
    assert np.array_equal(part, full[rows])


def test_gemm_rejects_bad_shapes():
    with pytest.raises(ValueError):
        oracle.gemm(np.zeros((3, 4)), np.zeros((5, 2)))


def test_normwise_error_definition():
    R = np.array([[3.0, 0.0], [0.0, 4.0]])
    X = R + np.array([[0.0, 0.5], [0.0, 0.0]])
    assert oracle.normwise_error(X, R) == pytest.approx(0.5 / 5.0, rel=1e-15)


# ----------------------------------------------------------------- bf16
def test_bf16_matches_torch_cast():
    r = _rng(20)
    x = np.concatenate([r.standard_normal(200000) * 10.0 ** r.integers(-30, 30, 200000),
                        [0.0, -0.0, 3.3895314e38, -3.3895314e38, 1e-40, -1e-42]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).float().numpy()
    got = P.bf16_rne(x)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def _golden_rounding():
    rows = []
    with open(os.path.join(GOLDEN, "rounding_cases.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, a, b = line.split()
                rows.append((k, float(a), float(b)))
    return rows


@pytest.mark.parametrize("kind,x,expect", _golden_rounding())
def test_rounding_golden(kind, x, expect):
    if kind == "bf16":
        assert float(P.bf16_rne(np.array([x], dtype=np.float32))[0]) == expect
    else:
        assert float(P.e4m3_rne_sat(np.float64(np.float32(x)))) == expect


def test_split_bound_and_exactness():
    r = _rng(21)
    a = (r.standard_normal(100000) * 10.0 ** r.integers(-5, 5, 100000)).astype(np.float32)
    hi, lo = P.split_bf16x3(a)
    # hi and lo are bf16 values
    assert np.array_equal(P.bf16_rne(hi), hi) and np.array_equal(P.bf16_rne(lo), lo)
    # |a - hi - lo| <= 2^-16 |a|: each RNE step keeps 8 significant bits
    err = np.abs(a.astype(np.float64) - hi.astype(np.float64) - lo.astype(np.float64))
    assert np.all(err <= 2.0 ** -16 * np.abs(a.astype(np.float64)))
    # values with at most 16 significant bits split exactly
    m = r.integers(-(2 ** 15), 2 ** 15, 10000).astype(np.float64) * 2.0 ** -10
    hi, lo = P.split_bf16x3(m.astype(np.float32))
    assert np.array_equal(hi.astype(np.float64) + lo.astype(np.float64), m)


def test_x3_expected_drops_only_lo_lo():
    # A = hiA + loA and B = hiB + loB with prescribed bf16 parts (integers times powers
    # of two): the full product minus the lo*lo term, computed in integers, must equal
    # the oracle's split product exactly.
    r = _rng(22)
    M, N, K = 19, 23, 40
    hiA_i = r.integers(128, 256, (M, K)) * r.choice([-1, 1], (M, K))   # 8 significant bits
    loA_i = r.integers(0, 128, (M, K))                                  # < half ulp of hi
    hiB_i = r.integers(128, 256, (K, N)) * r.choice([-1, 1], (K, N))
    loB_i = r.integers(0, 128, (K, N))
    # a = hi * 2^8 + lo (scaled by 2^-16 to keep it small); lo < 2^7 keeps RNE(a) == hi*2^8
    sc = 2.0 ** -16
    A = ((hiA_i * 256 + np.sign(hiA_i) * loA_i) * sc).astype(np.float32)
    B = ((hiB_i * 256 + np.sign(hiB_i) * loB_i) * sc).astype(np.float32)
    hA, lA = P.split_bf16x3(A)
    assert np.array_equal(hA.astype(np.float64), hiA_i * 256 * sc)
    exact_full = (A.astype(np.float64).astype(object) @ B.astype(np.float64).astype(object))
    la = (np.sign(hiA_i) * loA_i).astype(object)
    lb = (np.sign(hiB_i) * loB_i).astype(object)
    lolo = (la @ lb) * (sc * sc)
    expect = np.array(exact_full - lolo, dtype=np.float64)
    got = P.gemm_x3_expected(A, B, None, 1.0, 0.0)
    assert np.array_equal(got, expect)


# ----------------------------------------------------------------- e4m3
def _golden_points():
    out = []
    with open(os.path.join(GOLDEN, "e4m3_points.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                v, c = line.split()
                out.append((float(v), int(c, 16)))
    return out


@pytest.mark.parametrize("value,code", _golden_points())
def test_e4m3_golden_codes(value, code):
    assert int(P.e4m3_encode(np.float64(value))) == code
    assert float(P.e4m3_decode(np.uint8(code))) == value


def test_e4m3_matches_torch_in_range():
    r = _rng(23)
    x = (r.standard_normal(200000) * 10.0 ** r.integers(-4, 3, 200000)).astype(np.float32)
    x = x[np.abs(x) < 448.0]
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(P.e4m3_rne_sat(x), ref)


def test_e4m3_brute_force_nearest():
    # Nearest grid point by exhaustive search over all 254 finite codes; ties to even code.
    codes = np.arange(256, dtype=np.uint8)
    vals = P.e4m3_decode(codes)
    fin = ~np.isnan(vals)
    grid_vals, grid_codes = vals[fin], codes[fin]
    r = _rng(24)
    x = r.uniform(-460, 460, 3000)
    got = P.e4m3_rne_sat(x)
    for xi, gi in zip(x, got):
        d = np.abs(grid_vals - xi)
        best = d.min()
        cand = grid_codes[d == best]
        if len(cand) > 1:  # tie: even mantissa (low code bit 0)
            cand = cand[(cand & 1) == 0]
        expect = P.e4m3_decode(cand[0])
        if abs(xi) >= 448:
            expect = np.copysign(448.0, xi)
        assert gi == expect


def test_quantize_e4m3_bound_and_integers():
    A, _ = inputs.lowprec_inputs(300, 10, 260, seed=5)
    A = A.numpy()
    Q, S = P.quantize_tiles_e4m3(A)
    assert S.shape == (3, 3)
    D = P.dequantize_e4m3(Q, S)
    # each tile: |x - s q| <= s * 2^-4 * 2^floor(log2 |x/s|) (half spacing) or subnormal step
    for bi in range(3):
        for bj in range(3):
            blk = A[bi * 128:(bi + 1) * 128, bj * 128:(bj + 1) * 128].astype(np.float64)
            s = float(S[bi, bj])
            amax = np.abs(blk).max()
            assert np.frexp(s)[0] == 0.5 and 224.0 < amax / s <= 448.0   # power of two, top binade used
            y = np.abs(blk) / s
            half = np.where(y >= 2 ** -6, 2.0 ** (np.floor(np.log2(np.maximum(y, 1e-300))) - 4),
                            2.0 ** -10)
            err = np.abs(blk - D[bi * 128:(bi + 1) * 128, bj * 128:(bj + 1) * 128])
            assert np.all(err <= s * half * (1 + 2 ** -20) + 1e-300)
    # a tile whose amax is 448 has s = 1, and integers up to 16 are exact in e4m3
    I = np.random.default_rng(3).integers(-16, 17, (128, 128)).astype(np.float32)
    I[0, 0] = 448.0
    Q, S = P.quantize_tiles_e4m3(I)
    assert S[0, 0] == 1.0 and np.array_equal(P.dequantize_e4m3(Q, S), I.astype(np.float64))


def test_quantize_bf16_power_of_two_scales():
    A, _ = inputs.lowprec_inputs(200, 10, 150, seed=6)
    A = A.numpy()
    Q, S = P.quantize_tiles_bf16(A)
    for (bi, bj), s in np.ndenumerate(S):
        blk = A[bi * 128:(bi + 1) * 128, bj * 128:(bj + 1) * 128]
        amax = np.abs(blk).max()
        assert s >= amax and s / 2 < amax                   # s = 2^ceil(log2 amax)
        assert np.frexp(s)[0] == 0.5                        # a power of two
    D = P.dequantize_bf16(Q, S)
    # relative error of RNE to 8 significant bits
    assert np.all(np.abs(D - A) <= 2.0 ** -8 * np.abs(A) + 1e-30)


def test_lowprec_outlier_rows():
    A, B = inputs.lowprec_inputs(1000, 300, 500, seed=30)
    big_a = (A.abs().max(dim=1).values > 100).sum().item()
    big_b = (B.abs().max(dim=1).values > 100).sum().item()
    assert big_a == 10 and big_b == 5


def test_scaled_gemm_blockwise_form_brute_force():
    # The per-tile form, written as explicit loops over K scale blocks with the scale
    # indices (i // 128, kb) and (kb, j // 128), equals the dequantised product.
    r = _rng(25)
    M, N, K, t = 5, 7, 300, 128
    A = r.standard_normal((M, K)) * 10.0 ** r.integers(-2, 3, (M, K))
    B = r.standard_normal((K, N))
    QA, SA = P.quantize_tiles_e4m3(A.astype(np.float32))
    QB, SB = P.quantize_tiles_e4m3(B.astype(np.float32))
    qa, qb = P.e4m3_decode(QA), P.e4m3_decode(QB)
    brute = np.zeros((M, N))
    for i in range(M):
        for j in range(N):
            tot = 0.0
            for kb in range(-(-K // t)):
                part = sum(qa[i, k] * qb[k, j] for k in range(kb * t, min(K, kb * t + t)))
                tot += float(SA[i // t, kb]) * float(SB[kb, j // t]) * part
            brute[i, j] = tot
    got = P.gemm_scaled_expected(QA, SA, QB, SB, None, 1.0, 0.0, "fp8")
    assert np.allclose(got, brute, rtol=1e-12, atol=1e-12)


# ----------------------------------------------------------------- MLP (cost model)
from oracle import mlp as O  # noqa: E402


def _net(seed, dims):
    r = _rng(seed)
    return r.standard_normal(O.param_count(dims)) * 0.3


def test_mlp_gradients_match_central_differences():
    dims = [5, 7, 6, 1]
    p = _net(30, dims)
    r = _rng(31)
    X, y = r.standard_normal((9, 5)), r.standard_normal(9)
    _, g = O.gradients(p, dims, X, y)
    h = 1e-6
    num = np.empty_like(p)
    for i in range(len(p)):
        e = np.zeros_like(p)
        e[i] = h
        num[i] = (O.loss(p + e, dims, X, y) - O.loss(p - e, dims, X, y)) / (2 * h)
    assert np.max(np.abs(num - g)) <= 1e-7 * max(1.0, np.max(np.abs(g)))


def test_mlp_zero_weights_output_is_last_bias():
    dims = [4, 8, 8, 1]
    p = np.zeros(O.param_count(dims))
    p[-1] = 0.75
    out, _ = O.forward(p, dims, _rng(32).standard_normal((6, 4)))
    assert np.array_equal(out, np.full(6, 0.75))


def test_mlp_linear_layer_closed_form():
    # one linear layer: out = X w + b, dW = X^T dY with dY = 2 (out - y) / n
    r = _rng(33)
    dims = [3, 1]
    X, y = r.standard_normal((11, 3)), r.standard_normal(11)
    p = r.standard_normal(O.param_count(dims))
    L, g = O.gradients(p, dims, X, y)
    out = X @ p[:3] + p[3]
    dY = 2.0 * (out - y) / 11
    assert np.allclose(g[:3], X.T @ dY, rtol=1e-14, atol=1e-14)
    assert np.isclose(g[3], dY.sum(), rtol=1e-14, atol=1e-14)
    assert np.isclose(L, np.mean((out - y) ** 2), rtol=1e-14)


def test_adam_first_step_closed_form():
    # at step 1 the bias-corrected moments are g and g^2, so the update is
    # lr * g / (|g| + eps): a step of about lr against the sign of g
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    p, m, v = O.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, 0.01)
    assert np.allclose(p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


# ------------------------------------------------------------------ 3x3 convolution oracle
from oracle import conv as OC  # noqa: E402


def _int_conv_inputs(nb, H, W, cin, cout, seed):
    g = np.random.default_rng(seed)
    return (g.integers(-3, 4, (nb, H, W, cin)).astype(np.float64),
            g.integers(-3, 4, (3, 3, cin, cout)).astype(np.float64),
            g.integers(-3, 4, (nb, H, W, cout)).astype(np.float64))


def test_conv_brute_force_tiny():
    # every output element by its own six-deep loop, with the padding as an explicit bounds test
    X, Wt, Y0 = _int_conv_inputs(2, 3, 4, 2, 3, seed=61)
    nb, H, W, cin = X.shape
    cout = Wt.shape[3]
    ref = np.zeros((nb, H, W, cout))
    for n in range(nb):
        for y in range(H):
            for x in range(W):
                for co in range(cout):
                    s = 0.0
                    for dy in range(3):
                        for dx in range(3):
                            iy, ix = y + dy - 1, x + dx - 1
                            if 0 <= iy < H and 0 <= ix < W:
                                for ci in range(cin):
                                    s += X[n, iy, ix, ci] * Wt[dy, dx, ci, co]
                    ref[n, y, x, co] = 1.5 * s + 0.5 * Y0[n, y, x, co]
    np.testing.assert_array_equal(OC.conv3x3(X, Wt, Y0, 1.5, 0.5), ref)


def test_conv_center_tap_identity_is_copy():
    X, _, _ = _int_conv_inputs(2, 5, 6, 4, 4, seed=62)
    Wt = np.zeros((3, 3, 4, 4))
    Wt[1, 1] = np.eye(4)
    np.testing.assert_array_equal(OC.conv3x3(X, Wt), X)


def test_conv_delta_input_echoes_the_flipped_filter():
    # a single 1 at (n, y, x, c): output pixel (y + 1 - dy, x + 1 - dx) receives Wt[dy, dx, c, :]
    _, Wt, _ = _int_conv_inputs(1, 1, 1, 3, 5, seed=63)
    X = np.zeros((1, 6, 7, 3))
    X[0, 3, 2, 1] = 1.0
    Y = OC.conv3x3(X, Wt)
    expect = np.zeros_like(Y)
    for dy in range(3):
        for dx in range(3):
            expect[0, 3 + 1 - dy, 2 + 1 - dx] = Wt[dy, dx, 1]
    np.testing.assert_array_equal(Y, expect)


def test_conv_equals_gemm_on_explicit_im2col():
    # an independent construction: the im2col matrix built element by element, then the gemm oracle
    X, Wt, Y0 = _int_conv_inputs(2, 4, 5, 3, 6, seed=64)
    nb, H, W, cin = X.shape
    cols = np.zeros((nb * H * W, 9 * cin))
    for n in range(nb):
        for y in range(H):
            for x in range(W):
                for t in range(9):
                    iy, ix = y + t // 3 - 1, x + t % 3 - 1
                    if 0 <= iy < H and 0 <= ix < W:
                        cols[(n * H + y) * W + x, t * cin:(t + 1) * cin] = X[n, iy, ix]
    ref = oracle.gemm(cols, Wt.reshape(9 * cin, -1), Y0.reshape(nb * H * W, -1), 1.0, 2.0)
    np.testing.assert_array_equal(OC.conv3x3(X, Wt, Y0, 1.0, 2.0).reshape(nb * H * W, -1), ref)


def test_conv_pixel_subset_and_degenerate_scalars():
    X, Wt, Y0 = _int_conv_inputs(2, 4, 5, 3, 6, seed=65)
    full = OC.conv3x3(X, Wt, Y0, 1.0, 0.5).reshape(40, 6)
    pix = [0, 7, 19, 20, 39]
    np.testing.assert_array_equal(OC.conv3x3(X, Wt, Y0, 1.0, 0.5, pixels=pix), full[pix])
    # beta == 0 does not read Y0; alpha == 0 gives beta * Y0
    nan = np.full_like(Y0, np.nan)
    assert np.isfinite(OC.conv3x3(X, Wt, nan, 1.0, 0.0)).all()
    np.testing.assert_array_equal(OC.conv3x3(X, Wt, Y0, 0.0, 0.5), 0.5 * Y0)


# ---------------------------------------------------------------- back-to-back gemm oracle
from oracle import gemm2 as G2  # noqa: E402


def _int_chain(M, K, N1, N2, seed):
    g = np.random.default_rng(seed)
    return (g.integers(-4, 5, (M, K)).astype(np.float64), g.integers(-4, 5, (K, N1)).astype(np.float64),
            g.integers(-4, 5, (N1, N2)).astype(np.float64), g.integers(-4, 5, (M, N2)).astype(np.float64))


@pytest.mark.parametrize("relu", [False, True])
def test_gemm2_brute_force_tiny(relu):
    # every output element by explicit loops over both sums
    A, B, D, E0 = _int_chain(3, 4, 5, 2, seed=81)
    M, K = A.shape
    N1, N2 = D.shape
    ref = np.zeros((M, N2))
    for i in range(M):
        for j in range(N2):
            s = 0.0
            for h in range(N1):
                t = 0.0
                for k in range(K):
                    t += A[i, k] * B[k, h]
                if relu and t < 0:
                    t = 0.0
                s += t * D[h, j]
            ref[i, j] = 2.0 * s - 1.0 * E0[i, j]
    np.testing.assert_array_equal(G2.gemm2(A, B, D, E0, 2.0, -1.0, relu), ref)


def test_gemm2_identity_second_factor_is_the_gemm():
    # D = I without activation: E = alpha A B + beta E0, the gemm oracle's own loop
    A, B, _, E0 = _int_chain(6, 7, 5, 5, seed=82)
    np.testing.assert_array_equal(G2.gemm2(A, B, np.eye(5), E0, 1.5, 0.5), oracle.gemm(A, B, E0, 1.5, 0.5))


def test_gemm2_is_relu_between_two_gemm_oracle_calls():
    A, B, D, E0 = _int_chain(9, 8, 7, 6, seed=83)
    T = oracle.gemm(A, B)
    T[T < 0] = 0.0
    np.testing.assert_array_equal(G2.gemm2(A, B, D, E0, 1.0, 0.5, relu=True), oracle.gemm(T, D, E0, 1.0, 0.5))


def test_gemm2_closed_forms():
    A, B, D, E0 = _int_chain(5, 4, 3, 6, seed=84)
    # A B <= 0 everywhere (A >= 0, B <= 0): ReLU zeroes T, E = beta E0
    Ap, Bn = np.abs(A), -np.abs(B)
    np.testing.assert_array_equal(G2.gemm2(Ap, Bn, D, E0, 3.0, 0.5, relu=True), 0.5 * E0)
    # rank one: A = a 1^T, B = 1 b^T, D = d 1^T gives E = alpha * K (b . d) a 1^T
    a, b, d = np.arange(1.0, 6.0), np.arange(-1.0, 2.0), np.array([2.0, -1.0, 3.0])
    E = G2.gemm2(np.outer(a, np.ones(4)), np.outer(np.ones(4), b), np.outer(d, np.ones(6)), alpha=0.5)
    np.testing.assert_array_equal(E, 0.5 * 4 * np.dot(b, d) * np.outer(a, np.ones(6)))
    # beta == 0 does not read E0; row subset equals the rows of the full result
    assert np.isfinite(G2.gemm2(A, B, D, np.full_like(E0, np.nan), 1.0, 0.0)).all()
    full = G2.gemm2(A, B, D, E0, 1.0, 2.0, relu=True)
    np.testing.assert_array_equal(G2.gemm2(A, B, D, E0, 1.0, 2.0, relu=True, rows=[4, 0, 2]), full[[4, 0, 2]])
    # NaN in A B survives the ReLU
    An = A.copy()
    An[1, 0] = np.nan
    assert np.isnan(G2.gemm2(An, B, D, relu=True)[1]).all()


# ---------------------------------------------------------------- tensor contraction oracle
from oracle import contract as OT  # noqa: E402


def _int_tensor(shape, seed):
    return np.random.default_rng(seed).integers(-3, 4, shape).astype(np.float64)


def test_contract_brute_force_tiny():
    # C[x, a, b] = sum_c A[c, x, a] B[x, b, c] (batch x, row a, column b, contracted c), by loops
    X, Ad, Bd, Cd = 2, 3, 4, 5
    A = _int_tensor((Cd, X, Ad), 101)
    B = _int_tensor((X, Bd, Cd), 102)
    C0 = _int_tensor((X, Ad, Bd), 103)
    ref = np.zeros((X, Ad, Bd))
    for x in range(X):
        for a in range(Ad):
            for b in range(Bd):
                s = sum(A[c, x, a] * B[x, b, c] for c in range(Cd))
                ref[x, a, b] = 2.0 * s + 0.5 * C0[x, a, b]
    got = OT.contract(A, [7, 1, 3], B, [1, 4, 7], [1, 3, 4], C0, 2.0, 0.5)
    np.testing.assert_array_equal(got, ref)


def test_contract_matrix_and_batched_cases_are_gemms():
    A = _int_tensor((6, 5), 104)
    B = _int_tensor((5, 4), 105)
    C0 = _int_tensor((6, 4), 106)
    np.testing.assert_array_equal(OT.contract(A, [0, 1], B, [1, 2], [0, 2], C0, 1.5, -1.0),
                                  oracle.gemm(A, B, C0, 1.5, -1.0))
    # batch of 3 matrix products, batch mode leading in all three tensors
    Ab, Bb = _int_tensor((3, 6, 5), 107), _int_tensor((3, 5, 4), 108)
    got = OT.contract(Ab, [9, 0, 1], Bb, [9, 1, 2], [9, 0, 2])
    for t in range(3):
        np.testing.assert_array_equal(got[t], oracle.gemm(Ab[t], Bb[t]))


def test_contract_relabelled_output_is_a_transpose_and_beta_zero_skips_c0():
    A, B = _int_tensor((4, 3, 5), 109), _int_tensor((5, 2), 110)
    C = OT.contract(A, [0, 1, 2], B, [2, 3], [0, 1, 3])
    Ct = OT.contract(A, [0, 1, 2], B, [2, 3], [3, 1, 0])
    np.testing.assert_array_equal(Ct, np.transpose(C, (2, 1, 0)))
    assert np.isfinite(OT.contract(A, [0, 1, 2], B, [2, 3], [0, 1, 3], np.full((4, 3, 2), np.nan))).all()
    # no contracted mode: an outer product
    u, v = _int_tensor((4,), 111), _int_tensor((3,), 112)
    np.testing.assert_array_equal(OT.contract(u, [0], v, [1], [0, 1]), np.outer(u, v))


# ---------------------------------------------------------------- R x R convolution (R = 5, 7)
@pytest.mark.parametrize("R", [5, 7])
def test_conv2d_brute_force_tiny(R):
    g = np.random.default_rng(120 + R)
    X = g.integers(-3, 4, (2, 4, 5, 2)).astype(np.float64)
    Wt = g.integers(-3, 4, (R, R, 2, 3)).astype(np.float64)
    Y0 = g.integers(-3, 4, (2, 4, 5, 3)).astype(np.float64)
    P = R // 2
    nb, H, W, cin = X.shape
    ref = np.zeros((nb, H, W, 3))
    for n in range(nb):
        for y in range(H):
            for x in range(W):
                for co in range(3):
                    s = 0.0
                    for dy in range(R):
                        for dx in range(R):
                            iy, ix = y + dy - P, x + dx - P
                            if 0 <= iy < H and 0 <= ix < W:
                                for ci in range(cin):
                                    s += X[n, iy, ix, ci] * Wt[dy, dx, ci, co]
                    ref[n, y, x, co] = -1.0 * s + 0.5 * Y0[n, y, x, co]
    np.testing.assert_array_equal(OC.conv2d(X, Wt, Y0, -1.0, 0.5), ref)


@pytest.mark.parametrize("R", [5, 7, 11])
def test_conv2d_center_tap_and_delta(R):
    g = np.random.default_rng(130 + R)
    X = g.integers(-3, 4, (1, 6, 7, 3)).astype(np.float64)
    Wt = np.zeros((R, R, 3, 3))
    Wt[R // 2, R // 2] = np.eye(3)
    np.testing.assert_array_equal(OC.conv2d(X, Wt), X)
    # a single 1 at (y0, x0, c): output pixel (y0 + P - dy, x0 + P - dx) receives Wt[dy, dx, c, :]
    Wr = g.integers(-3, 4, (R, R, 3, 4)).astype(np.float64)
    D = np.zeros((1, 13, 12, 3))
    y0, x0, P = 6, 5, R // 2
    D[0, y0, x0, 2] = 1.0
    Y = OC.conv2d(D, Wr)
    expect = np.zeros_like(Y)
    for dy in range(R):
        for dx in range(R):
            yy, xx = y0 + P - dy, x0 + P - dx
            if 0 <= yy < 13 and 0 <= xx < 12:
                expect[0, yy, xx] = Wr[dy, dx, 2]
    np.testing.assert_array_equal(Y, expect)


def test_conv2d_equals_gemm_on_explicit_im2col_r5():
    g = np.random.default_rng(140)
    X = g.integers(-3, 4, (2, 5, 6, 3)).astype(np.float64)
    Wt = g.integers(-3, 4, (5, 5, 3, 4)).astype(np.float64)
    nb, H, W, cin = X.shape
    cols = np.zeros((nb * H * W, 25 * cin))
    for n in range(nb):
        for y in range(H):
            for x in range(W):
                for t in range(25):
                    iy, ix = y + t // 5 - 2, x + t % 5 - 2
                    if 0 <= iy < H and 0 <= ix < W:
                        cols[(n * H + y) * W + x, t * cin:(t + 1) * cin] = X[n, iy, ix]
    ref = oracle.gemm(cols, Wt.reshape(25 * cin, -1))
    np.testing.assert_array_equal(OC.conv2d(X, Wt).reshape(nb * H * W, -1), ref)
