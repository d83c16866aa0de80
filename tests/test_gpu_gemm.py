"""GPU parity of tgemm (F32 and split-bf16x3) against the FP64 oracle.

Operation: C = alpha*A*B + beta*C (Tiramisu paper, Section I).  Every call
goes through the C ABI (libtgemm.so) via the thin ctypes binding.

Bars: bit-exact on small-integer inputs (every product and partial sum is an
integer below 2^24, so any summation order gives the exact result); normwise
relative error <= 1e-5 for F32 and x3 on U[-1, 1] inputs.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import precision as P
from paper_1804_10694_amd import inputs

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
TOL = 1e-5


@pytest.fixture(scope="module")
def tg():
    from paper_1804_10694_amd import tgemm
    tgemm.set_policy("default")
    return tgemm


def _run(tg, A, B, C0, alpha, beta, dtype, sid=None, group_m=8, xcd=1, ld_pad=0):
    """Runs one gemm on the GPU, optionally with padded leading dimensions and NaN
    canaries around every matrix; returns (C, canaries_intact)."""
    M, K = A.shape
    N = B.shape[1]
    if ld_pad:
        # ld_pad == "align4": each row stride rounded up to a multiple of 4 elements, plus 4
        def extra(cols):
            return ((-cols) % 4) + 4 if ld_pad == "align4" else ld_pad
        Ab, _ = inputs.padded(A, extra(K))
        Bb, _ = inputs.padded(B, extra(N))
        Cb, _ = inputs.padded(C0, extra(N))
        Ad, Bd, Cd = Ab.to(DEV), Bb.to(DEV), Cb.to(DEV)
        a, b, c = Ad[:, :K], Bd[:, :N], Cd[:, :N]
    else:
        Ad, Bd, Cd = A.to(DEV), B.to(DEV), C0.clone().to(DEV)
        a, b, c = Ad, Bd, Cd
    if sid is None:
        tg.gemm(a, b, c, alpha, beta, dtype)
    else:
        tg.gemm_with_schedule(a, b, c, alpha, beta, dtype, sid, group_m, xcd)
    torch.cuda.synchronize()
    ok = True
    if ld_pad:
        ok = bool(torch.isnan(Cd[:, N:]).all().item())
    return c.cpu(), ok


def _serving(tg, dtype, vec=None):
    out = []
    for sid, info in tg.schedules(dtype):
        if vec is None or info["vec"] == vec:
            out.append((sid, info))
    return out


# ------------------------------------------------------------ exact (integers)
@pytest.mark.parametrize("dtype", ["f32", "x3"])
def test_every_schedule_bit_exact_on_integers(tg, dtype):
    # Ragged in every dimension: several tiles plus partial tiles and a K remainder.
    M, N, K = 300, 200, 100
    A, B, C0 = inputs.integer_inputs(M, N, K, seed=7)
    for alpha, beta in [(1.0, 0.5), (1.5, 0.0)]:
        ref = oracle.gemm(A, B, C0, alpha, beta)
        for sid, info in _serving(tg, dtype):
            pad = 0 if info["vec"] == 4 else 3   # vec=1 schedules also get odd strides
            for gm, xcd in [(8, 1), (1, 0)]:
                print(f"schedule {sid} {info} alpha={alpha} beta={beta} gm={gm} xcd={xcd}",
                      flush=True)
                got, ok = _run(tg, A, B, C0, alpha, beta, dtype, sid, gm, xcd, ld_pad=pad)
                assert ok, f"canary overwritten by schedule {sid}"
                np.testing.assert_array_equal(got.numpy().astype(np.float64), ref,
                                              err_msg=f"schedule {sid} {info}")


@pytest.mark.parametrize("dtype", ["f32", "x3"])
def test_aligned_multi_tile_exact(tg, dtype):
    M, N, K = 512, 512, 256   # full tiles only for every schedule
    A, B, C0 = inputs.integer_inputs(M, N, K, seed=8)
    ref = oracle.gemm(A, B, C0, 1.0, 0.5)
    for sid, info in _serving(tg, dtype, vec=4):
        got, _ = _run(tg, A, B, C0, 1.0, 0.5, dtype, sid)
        np.testing.assert_array_equal(got.numpy().astype(np.float64), ref,
                                      err_msg=f"schedule {sid} {info}")


@pytest.mark.parametrize("dtype", ["f32", "x3"])
def test_packed_schedules_exact_with_vector_packing(tg, dtype):
    # Rows whose strides allow the packing pass's 16-byte loads (the "align4" padding),
    # ragged in M and N, K = 100 (the last group of 8 k falls back to element loads) and
    # K = 96 (every group is a vector load), with NaN canaries around every matrix.
    for (M, N, K) in [(300, 200, 100), (260, 130, 96)]:
        A, B, C0 = inputs.integer_inputs(M, N, K, seed=12 + K)
        ref = oracle.gemm(A, B, C0, 1.0, 0.5)
        for sid, info in _serving(tg, dtype, vec=0):
            print(f"packed schedule {sid} {info} M={M} N={N} K={K}", flush=True)
            got, ok = _run(tg, A, B, C0, 1.0, 0.5, dtype, sid, ld_pad="align4")
            assert ok, f"canary overwritten by schedule {sid}"
            np.testing.assert_array_equal(got.numpy().astype(np.float64), ref,
                                          err_msg=f"schedule {sid} {info} {(M, N, K)}")


@pytest.mark.parametrize("dtype", ["f32", "x3"])
def test_inplace_schedules_exact_off_alignment(tg, dtype):
    # In-place schedules load 16 bytes at any 4-byte aligned address: operands are views
    # one float into NaN-filled buffers (bases and rows off 16-byte alignment), K and N
    # off a multiple of 4 (the tail units switch to 4-byte loads), ragged M and N over
    # several tiles, both tile orders; the NaNs around the operands must never be read.
    for (M, N, K) in [(300, 270, 37), (200, 130, 129), (129, 67, 300)]:
        A, B, C0 = inputs.integer_inputs(M, N, K, seed=60 + K)
        ref = oracle.gemm(A, B, C0, 1.0, 0.5)
        Ab = torch.full((M + 1, K + 5), float("nan"))
        Bb = torch.full((K + 1, N + 3), float("nan"))
        Ab[1:, 1:K + 1] = A
        Bb[1:, 1:N + 1] = B
        Ad, Bd = Ab.to(DEV), Bb.to(DEV)
        a, b = Ad[1:, 1:K + 1], Bd[1:, 1:N + 1]
        for sid, info in _serving(tg, dtype):
            if not info["inplace"]:
                continue
            for gm, xcd in [(8, 0), (1, 1)]:
                print(f"in-place schedule {sid} {info} {(M, N, K)} gm={gm} xcd={xcd}", flush=True)
                c = C0.clone().to(DEV)
                tg.gemm_with_schedule(a, b, c, 1.0, 0.5, dtype, sid, gm, xcd)
                torch.cuda.synchronize()
                np.testing.assert_array_equal(c.cpu().numpy().astype(np.float64), ref,
                                              err_msg=f"schedule {sid} {info} {(M, N, K)}")


@pytest.mark.parametrize("dtype,K", [("f32", 1024), ("x3", 2048)])
def test_packed_schedules_exact_padded_row_pitch(tg, dtype, K):
    # K * element size a multiple of 4 KB: the packed rows get 512 bytes of padding past K,
    # so every panel load runs on the padded pitch; ragged M and N, NaN canaries around C
    M, N = 300, 270
    A, B, C0 = inputs.integer_inputs(M, N, K, seed=40 + K)
    ref = oracle.gemm(A, B, C0, 1.0, 0.5)
    for sid, info in _serving(tg, dtype, vec=0):
        print(f"packed schedule {sid} {info} M={M} N={N} K={K}", flush=True)
        got, ok = _run(tg, A, B, C0, 1.0, 0.5, dtype, sid, ld_pad="align4")
        assert ok, f"canary overwritten by schedule {sid}"
        np.testing.assert_array_equal(got.numpy().astype(np.float64), ref,
                                      err_msg=f"schedule {sid} {info} {(M, N, K)}")


def test_brute_force_tiny_sizes(tg):
    # All small (M, N) with a ladder of K values, default policy, integer inputs.
    Ks = [1, 2, 3, 5, 7, 8, 9, 15, 16, 17, 31, 32, 33, 63, 64, 65, 127, 128, 129]
    for M in (1, 2, 3, 7, 16, 31, 32, 33):
        for N in (1, 2, 5, 17, 32, 33):
            for K in Ks:
                A, B, C0 = inputs.integer_inputs(M, N, K, seed=M * 1000 + N * 10 + K)
                ref = oracle.gemm(A, B, C0, 1.0, 0.5)
                for dtype in ("f32", "x3"):
                    got, ok = _run(tg, A, B, C0, 1.0, 0.5, dtype, ld_pad=3)
                    assert ok
                    np.testing.assert_array_equal(got.numpy().astype(np.float64), ref,
                                                  err_msg=f"{dtype} M={M} N={N} K={K}")


def test_x3_drops_only_lo_lo_term(tg):
    # Integers in [-512, 512] are not all bf16 values: a = hi + lo with |lo| <= 2.
    # Products stay below 2^24, so the GPU sum is exact and must equal the oracle's
    # split product hi*hi + hi*lo + lo*hi, and differ from the exact product.
    g = torch.Generator().manual_seed(9)
    M, N, K = 130, 70, 40
    A = torch.randint(-512, 513, (M, K), generator=g).float()
    B = torch.randint(-512, 513, (K, N), generator=g).float()
    C0 = torch.zeros(M, N)
    expect = P.gemm_x3_expected(A.numpy(), B.numpy(), None, 1.0, 0.0)
    exact = oracle.gemm(A, B, None, 1.0, 0.0)
    got, _ = _run(tg, A, B, C0, 1.0, 0.0, "x3")
    np.testing.assert_array_equal(got.numpy().astype(np.float64), expect)
    assert not np.array_equal(expect, exact)
    # plain F32 gives the exact product on the same inputs
    got32, _ = _run(tg, A, B, C0, 1.0, 0.0, "f32")
    np.testing.assert_array_equal(got32.numpy().astype(np.float64), exact)


# ------------------------------------------------------------ tolerance
@pytest.mark.parametrize("dtype", ["f32", "x3"])
def test_config_sgemm_256(tg, dtype):
    # 256^3, U[-1,1] from seed 1, alpha = 1.5, beta = 0.5
    A, B, C0 = inputs.gemm_inputs(256, 256, 256, seed=1)
    ref = oracle.gemm(A, B, C0, 1.5, 0.5)
    got, _ = _run(tg, A, B, C0, 1.5, 0.5, dtype)
    err = oracle.normwise_error(got.numpy(), ref)
    print(f"{dtype} 256^3 normwise error {err:.3e}")
    assert err <= TOL
    if dtype == "x3":
        assert err <= 8e-6   # expected magnitude of the split product (~4e-6)


@pytest.mark.parametrize("dtype", ["f32", "x3"])
def test_every_schedule_within_tolerance_ragged(tg, dtype):
    M, N, K = 517, 389, 301
    A, B, C0 = inputs.gemm_inputs(M, N, K, seed=10)
    ref = oracle.gemm(A, B, C0, 1.0, 1.0)
    for sid, info in _serving(tg, dtype):
        pad = "align4" if info["vec"] == 4 else 1
        got, ok = _run(tg, A, B, C0, 1.0, 1.0, dtype, sid, ld_pad=pad)
        assert ok
        err = oracle.normwise_error(got.numpy(), ref)
        assert err <= TOL, f"schedule {sid} {info}: {err}"


def test_degenerate_cases(tg):
    M, N, K = 70, 90, 50
    A, B, C0 = inputs.gemm_inputs(M, N, K, seed=11)
    for dtype in ("f32", "x3"):
        # beta == 0 never reads C: NaN in the old C must vanish
        Cn = torch.full((M, N), float("nan"))
        got, _ = _run(tg, A, B, Cn, 1.0, 0.0, dtype)
        assert not torch.isnan(got).any()
        assert oracle.normwise_error(got.numpy(), oracle.gemm(A, B, None, 1.0, 0.0)) <= TOL
        # alpha == 0: C = beta*C, A and B not read (NaN in them must not matter)
        An = torch.full((M, K), float("nan"))
        got, _ = _run(tg, An, B, C0, 0.0, 0.5, dtype)
        np.testing.assert_array_equal(got.numpy(), (0.5 * C0).numpy())
        # K == 0: C = beta*C
        got, _ = _run(tg, torch.zeros(M, 0), torch.zeros(0, N), C0, 1.0, 2.0, dtype)
        np.testing.assert_array_equal(got.numpy(), (2.0 * C0).numpy())
        # alpha == 0 and beta == 0: zeros, even over NaN
        got, _ = _run(tg, A, B, Cn, 0.0, 0.0, dtype)
        assert (got == 0).all()
        # M == 0 / N == 0: nothing launched, nothing to check beyond success
        tg.gemm(torch.zeros(0, K, device=DEV), B.to(DEV), torch.zeros(0, N, device=DEV), 1.0, 0.0,
                dtype)


def test_deterministic_repeats(tg):
    A, B, C0 = inputs.gemm_inputs(600, 500, 700, seed=12)
    for dtype in ("f32", "x3"):
        r1, _ = _run(tg, A, B, C0, 1.0, 1.0, dtype)
        r2, _ = _run(tg, A, B, C0, 1.0, 1.0, dtype)
        assert torch.equal(r1, r2)


def test_linearity_and_k_split(tg):
    M, N, K = 260, 190, 330
    A, B, C0 = inputs.gemm_inputs(M, N, K, seed=13)
    ref = oracle.gemm(A, B, C0, 1.0, 1.0)
    for dtype in ("f32", "x3"):
        # C0 + A[:, :K1] B[:K1] then + A[:, K1:] B[K1:] equals one call within tolerance
        K1 = 147
        Cd = C0.clone().to(DEV)
        Ad, Bd = A.to(DEV), B.to(DEV)
        tg.gemm(Ad[:, :K1].contiguous(), Bd[:K1].contiguous(), Cd, 1.0, 1.0, dtype)
        tg.gemm(Ad[:, K1:].contiguous(), Bd[K1:].contiguous(), Cd, 1.0, 1.0, dtype)
        torch.cuda.synchronize()
        assert oracle.normwise_error(Cd.cpu().numpy(), ref) <= TOL


def test_rejects_host_tensors(tg):
    A = torch.zeros(4, 4)
    with pytest.raises(ValueError):
        tg.gemm(A, A, A, 1.0, 0.0, "f32")


# ------------------------------------------------------------ full sizes, sampled
def _sampled_rows(M, seed, count=12):
    r = np.random.default_rng(seed)
    rows = set(r.choice(M, size=count, replace=False).tolist())
    rows.update([0, M - 1])              # the last row sits in a partial tile when M % BM != 0
    return np.array(sorted(rows))


@pytest.mark.parametrize("shape,seed", [((8192, 8192, 8192), 2), ((4097, 3001, 2053), 3)])
def test_full_size_configs_sampled(tg, shape, seed):
    # The benchmark shapes under the default policy (the launch configuration the benchmark
    # times); the oracle computes a sample of whole rows.
    M, N, K = shape
    A, B, C0 = inputs.gemm_inputs(M, N, K, seed)
    rows = _sampled_rows(M, seed)
    ref = oracle.gemm_rows(A, B, C0, 1.0, 1.0, rows)
    Ad, Bd = A.to(DEV), B.to(DEV)
    for dtype in ("f32", "x3"):
        Cd = C0.to(DEV)
        tg.gemm(Ad, Bd, Cd, 1.0, 1.0, dtype)
        torch.cuda.synchronize()
        got = Cd[torch.from_numpy(rows).to(DEV)].cpu().numpy()
        err = oracle.normwise_error(got, ref)
        print(f"{dtype} {shape} sampled-row normwise error {err:.3e}")
        assert err <= TOL
        del Cd


def test_deep_k_beyond_packed_reach(tg):
    # K = 2^21 + 3: a 256-row packed f32 tile would span more than 2^31 bytes, past
    # the 32-bit offsets of the buffer loads.  A forced packed schedule is refused
    # (no launch); the default rule takes a direct schedule, exact on integer inputs.
    M, N, K = 8, 8, (1 << 21) + 3
    g = torch.Generator().manual_seed(41)
    A = torch.randint(-2, 3, (M, K), generator=g).float()
    B = torch.randint(-2, 3, (K, N), generator=g).float()
    C0 = torch.zeros(M, N)
    ref = oracle.gemm(A, B, C0, 1.0, 0.0)   # |partial sums| <= 4 * 2^21 < 2^24: exact
    packed = [sid for sid, info in _serving(tg, "f32", vec=0)]
    Ad, Bd, Cd = A.to(DEV), B.to(DEV), C0.to(DEV)
    with pytest.raises(tg.TgemmError):
        tg.gemm_with_schedule(Ad, Bd, Cd, 1.0, 0.0, "f32", packed[0], 8, 1)
    tg.gemm(Ad, Bd, Cd, 1.0, 0.0, "f32")
    torch.cuda.synchronize()
    np.testing.assert_array_equal(Cd.cpu().numpy().astype(np.float64), ref)


@pytest.mark.parametrize("ldc", [(1 << 25) - 8, (1 << 25) + 8], ids=["ldc_below_2^25", "ldc_above_2^25"])
@pytest.mark.parametrize("dtype", ["f32", "x3"])
def test_epilogue_row_pitch_near_32bit_offsets(tg, dtype, ldc):
    # The epilogue reaches C through 32-bit buffer offsets below a row pitch of 2^25
    # elements and through a plain per-element loop from 2^25 on; both must write
    # exactly the M x N elements (NaN canaries in the rest of each row stay).
    M, N, K = 3, 50, 40
    A, B, C0 = inputs.integer_inputs(M, N, K, seed=42)
    ref = oracle.gemm(A, B, C0, 1.5, 0.5)
    store = torch.full((M, ldc), float("nan"), device=DEV)
    C = store[:, :N]
    C.copy_(C0.to(DEV))
    tg.gemm(A.to(DEV), B.to(DEV), C, 1.5, 0.5, dtype)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(C.cpu().numpy().astype(np.float64), ref)
    assert bool(torch.isnan(store[:, N:N + 1024]).all().item())
    assert bool(torch.isnan(store[:, -1024:]).all().item())
    del store
    torch.cuda.empty_cache()
