"""GPU parity of the grouped persistent gemm (tgemm_batched) and its HIP-graph replay.

Every problem p of a set must satisfy C_p = alpha_p A_p B_p + beta_p C_p
(Tiramisu paper, Section I) to the same bars as the one-problem kernels:
bit-exact on integer inputs, normwise <= 1e-5 on U[-1, 1] inputs.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1804_10694_amd import inputs

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def tg():
    from paper_1804_10694_amd import tgemm
    yield tgemm
    tgemm.shutdown()


def _problem_set(dims, seed_base, integer=False):
    host = []
    for p, (m, n, k) in enumerate(dims):
        if integer:
            host.append(inputs.integer_inputs(int(m), int(n), int(k), seed_base + p))
        else:
            host.append(inputs.gemm_inputs(int(m), int(n), int(k), seed_base + p))
    return host


NEVER = 2**31 - 1
# plan shapes: the default (tuned or built-in); direct tiles only (mixed, all 128, all 64);
# packed 256 x 256 tiles for the larger problems; packed tiles for every problem
SHAPES = [None, {"threshold": 96, "large": NEVER}, {"threshold": 0, "large": NEVER},
          {"threshold": NEVER, "large": NEVER}, {"threshold": 96, "large": 200},
          {"threshold": NEVER, "large": 0}]
SHAPE_IDS = ["default", "direct-mixed", "direct-128", "direct-64", "hybrid", "packed-all"]


def _run_batched(tg, host, alphas, betas, dtype, shape=None):
    As = [h[0].to(DEV) for h in host]
    Bs = [h[1].to(DEV) for h in host]
    Cs = [h[2].clone().to(DEV) for h in host]
    tg.gemm_batched(As, Bs, Cs, alphas, betas, dtype, shape=shape)
    torch.cuda.synchronize()
    return [c.cpu() for c in Cs]


@pytest.mark.parametrize("shape", SHAPES, ids=SHAPE_IDS)
@pytest.mark.parametrize("dtype", ["f32", "x3"])
def test_small_set_bit_exact_on_integers(tg, dtype, shape):
    rng = np.random.default_rng(51)
    dims = rng.integers(1, 300, size=(60, 3))
    dims[3] = (0, 5, 7)          # empty problems launch nothing
    dims[4] = (6, 0, 9)
    dims[5] = (17, 33, 0)        # K == 0: C = beta*C
    dims[6] = (128, 128, 64)     # full tiles only
    dims[7] = (256, 130, 96)     # 128-tile config with an edge
    host = _problem_set(dims, 5000, integer=True)
    alphas = [1.5 if p % 2 else 1.0 for p in range(len(dims))]
    betas = [0.5 if p % 3 else 0.0 for p in range(len(dims))]
    print(f"{dtype} shape {shape}", flush=True)
    got = _run_batched(tg, host, alphas, betas, dtype, shape)
    for p, (h, g) in enumerate(zip(host, got)):
        ref = oracle.gemm(h[0], h[1], h[2], alphas[p], betas[p])
        np.testing.assert_array_equal(g.numpy().astype(np.float64), ref, err_msg=f"problem {p} {dims[p]}")


@pytest.mark.parametrize("large", [0, NEVER])
def test_alpha_zero_and_padded_strides(tg, large):
    # alpha == 0 must not read A (NaN there), and row strides wider than the matrices
    # (unaligned and aligned) take the 4-byte and 16-byte load configurations.
    dims = [(40, 50, 30), (200, 160, 120), (129, 257, 65), (96, 96, 96)]
    host = _problem_set(dims, 5100)
    As, Bs, Cs, views = [], [], [], []
    for p, (A, B, C0) in enumerate(host):
        pad = 3 if p % 2 else 4
        Ab, _ = inputs.padded(A, pad)
        Bb, _ = inputs.padded(B, pad)
        Cb, _ = inputs.padded(C0, pad)
        Ad, Bd, Cd = Ab.to(DEV), Bb.to(DEV), Cb.to(DEV)
        As.append(Ad[:, :A.shape[1]])
        Bs.append(Bd[:, :B.shape[1]])
        Cs.append(Cd[:, :C0.shape[1]])
        views.append(Cd)
    As[0] = torch.full_like(As[0], float("nan"))
    alphas, betas = [0.0, 1.0, 1.0, 2.0], [0.5, 0.5, 0.0, 1.0]
    tg.gemm_batched(As, Bs, Cs, alphas, betas, "f32", shape={"threshold": 96, "large": large})
    torch.cuda.synchronize()
    np.testing.assert_array_equal(Cs[0].cpu().numpy(), (0.5 * host[0][2]).numpy())
    for p in range(1, 4):
        ref = oracle.gemm(host[p][0], host[p][1], host[p][2], alphas[p], betas[p])
        assert oracle.normwise_error(Cs[p].cpu().numpy(), ref) <= 1e-5
        assert torch.isnan(views[p][:, host[p][2].shape[1]:]).all()    # canaries intact


# in-place class (64 x 64 tiles, panels of 16).  16-byte loads: K and N multiples of 4 on
# 16-byte aligned rows; K below, at and past one panel, ragged M and N, one-row and one-unit
# problems.  4-byte loads: any K and N, rows at any 4-byte offset.
INPLACE_DIMS = [(1, 4, 4), (65, 68, 20), (130, 132, 36), (64, 64, 64), (200, 100, 100),
                (17, 260, 8), (129, 4, 516), (300, 300, 12), (3, 76, 1000)]
INPLACE_DIMS_ODD = [(1, 1, 1), (5, 7, 3), (65, 67, 21), (131, 129, 37), (70, 3, 517), (64, 64, 17),
                    (33, 250, 15), (250, 33, 31), (2, 130, 1001)]


# tile threshold NEVER: every problem on 64 x 64 in-place tiles; 0: every one on 128 x 128
IP_TILE = {64: {"threshold": NEVER, "large": NEVER}, 128: {"threshold": 0, "large": NEVER}}


@pytest.mark.parametrize("tile", [64, 128])
@pytest.mark.parametrize("pad", [4, 3], ids=["vec16", "vec4"])
@pytest.mark.parametrize("dims", [INPLACE_DIMS, INPLACE_DIMS_ODD], ids=["aligned", "odd"])
@pytest.mark.parametrize("dtype", ["f32", "x3"])
def test_inplace_tiles_bit_exact_with_nan_padding(tg, dtype, dims, pad, tile):
    # All problems take the in-place tiles of one size.  A and B sit in buffers
    # `pad` (or pad + 4) columns wider than the matrices, the extra columns NaN: A past K
    # (the row's tail) must read as zero, and B's columns past N only reach accumulator
    # columns that are never stored.  C's canary columns must stay NaN.  Odd dimensions
    # and a pad of 3 put rows off 16-byte alignment: the tiles take 16-byte loads at those
    # 4-byte aligned addresses (exactness here pins that the hardware honours them), with
    # 4-byte loads for A's tail panel when K % 4 != 0 and for the panel holding B's last
    # row on edge tiles when N % 4 != 0.
    host = _problem_set(dims, 5400, integer=True)
    As, Bs, Cs, views = [], [], [], []
    for p, (A, B, C0) in enumerate(host):
        pad = pad if p % 2 else pad + 4
        Ab, _ = inputs.padded(A, pad)
        Bb, _ = inputs.padded(B, pad)
        Cb, _ = inputs.padded(C0, 3)
        Ad, Bd, Cd = Ab.to(DEV), Bb.to(DEV), Cb.to(DEV)
        As.append(Ad[:, :A.shape[1]])
        Bs.append(Bd[:, :B.shape[1]])
        Cs.append(Cd[:, :C0.shape[1]])
        views.append(Cd)
    alphas = [1.5 if p % 2 else 1.0 for p in range(len(host))]
    betas = [0.5 if p % 3 else 0.0 for p in range(len(host))]
    print(f"in-place {tile} {dtype} pad {pad}", flush=True)
    tg.gemm_batched(As, Bs, Cs, alphas, betas, dtype, shape=IP_TILE[tile])
    torch.cuda.synchronize()
    for p, h in enumerate(host):
        ref = oracle.gemm(h[0], h[1], h[2], alphas[p], betas[p])
        np.testing.assert_array_equal(Cs[p].cpu().numpy().astype(np.float64), ref,
                                      err_msg=f"problem {p} {dims[p]}")
        assert torch.isnan(views[p][:, h[2].shape[1]:]).all()


@pytest.mark.parametrize("tile", [64, 128])
@pytest.mark.parametrize("dims", [INPLACE_DIMS, INPLACE_DIMS_ODD], ids=["aligned", "odd"])
@pytest.mark.parametrize("dtype", ["f32", "x3"])
def test_inplace_tiles_uniform_inputs(tg, dtype, dims, tile):
    host = _problem_set(dims, 5500)
    alphas, betas = [1.0] * len(host), [1.0] * len(host)
    got = _run_batched(tg, host, alphas, betas, dtype, IP_TILE[tile])
    for p, (h, g) in enumerate(zip(host, got)):
        ref = oracle.gemm(h[0], h[1], h[2], 1.0, 1.0)
        assert oracle.normwise_error(g.numpy(), ref) <= 1e-5, f"problem {p} {dims[p]}"


@pytest.mark.parametrize("shape", [None, {"threshold": NEVER, "large": NEVER}], ids=["default", "inplace-64"])
@pytest.mark.parametrize("dtype", ["f32", "x3"])
def test_grouped_config_512_problems(tg, dtype, shape):
    # 512 problems, M, N, K log-uniform in [16, 2048] (seed 4), matrices from seeds
    # 4000 + p, alpha = 1, beta = 0.5.
    dims = inputs.grouped_dims()
    host = _problem_set(dims, 4000)
    alphas, betas = [1.0] * len(dims), [0.5] * len(dims)
    got = _run_batched(tg, host, alphas, betas, dtype, shape)
    worst = 0.0
    for p, (h, g) in enumerate(zip(host, got)):
        ref = oracle.gemm(h[0], h[1], h[2], 1.0, 0.5)
        worst = max(worst, oracle.normwise_error(g.numpy(), ref))
    print(f"{dtype}: worst per-problem normwise error over 512 problems {worst:.3e}")
    assert worst <= 1e-5


@pytest.mark.parametrize("dtype", ["f32", "x3"])
def test_grouped_config_512_tuned_plan_graph_replay(tg, dtype):
    # The 512-problem set as the benchmark runs it: plan shape tuned on the set, plan
    # built by one eager call, the launch captured in a HIP graph and replayed.  C is
    # restored between replays (eager copies), so every replay is checked against the
    # same oracle result; replays must also agree bit for bit.
    dims = inputs.grouped_dims()
    host = _problem_set(dims, 4000)
    alphas, betas = [1.0] * len(dims), [0.5] * len(dims)
    As = [h[0].to(DEV) for h in host]
    Bs = [h[1].to(DEV) for h in host]
    C0 = [h[2].to(DEV) for h in host]
    Cs = [c.clone() for c in C0]
    shape = tg.gemm_batched_autotune(As, Bs, Cs, alphas, betas, dtype, reps=3)
    print(f"{dtype}: tuned plan shape {shape}", flush=True)
    tg.gemm_batched(As, Bs, Cs, alphas, betas, dtype)      # plans
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        tg.gemm_batched(As, Bs, Cs, alphas, betas, dtype)
    refs = [oracle.gemm(h[0], h[1], h[2], 1.0, 0.5) for h in host]
    first = None
    for r in range(3):
        for c, c0 in zip(Cs, C0):
            c.copy_(c0)
        graph.replay()
        torch.cuda.synchronize()
        got = [c.cpu() for c in Cs]
        worst = max(oracle.normwise_error(g.numpy(), ref) for g, ref in zip(got, refs))
        print(f"{dtype} replay {r}: worst per-problem normwise error {worst:.3e}", flush=True)
        assert worst <= 1e-5
        if first is None:
            first = got
        else:
            for p in range(len(dims)):
                assert torch.equal(got[p], first[p]), f"replay {r} problem {p}"
    del graph


@pytest.mark.parametrize("large", [200, NEVER])
def test_graph_capture_replays_match_eager(tg, large):
    rng = np.random.default_rng(52)
    dims = rng.integers(16, 400, size=(40, 3))
    host = _problem_set(dims, 5200)
    alphas, betas = [1.0] * 40, [0.5] * 40
    As = [h[0].to(DEV) for h in host]
    Bs = [h[1].to(DEV) for h in host]
    Cg = [h[2].clone().to(DEV) for h in host]        # graph-updated
    Ce = [h[2].clone().to(DEV) for h in host]        # eager-updated
    shape = {"threshold": 96, "large": large}
    # plan exists before capture (first call plans; it also advances Cg once)
    tg.gemm_batched(As, Bs, Cg, alphas, betas, "x3", shape=shape)
    tg.gemm_batched(As, Bs, Ce, alphas, betas, "x3", shape=shape)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        tg.gemm_batched(As, Bs, Cg, alphas, betas, "x3", shape=shape)
    for r in range(3):
        graph.replay()
        tg.gemm_batched(As, Bs, Ce, alphas, betas, "x3", shape=shape)
        torch.cuda.synchronize()
        for p in range(40):
            assert torch.equal(Cg[p], Ce[p]), f"replay {r} problem {p}"


def test_capture_without_plan_is_refused(tg):
    A = torch.rand(33, 44, device=DEV)
    B = torch.rand(44, 55, device=DEV)
    C = torch.rand(33, 55, device=DEV)
    arr = lambda t, v: (t * len(v))(*v)                      # noqa: E731
    i64, p = ctypes.c_int64, ctypes.c_void_p
    args = (1, arr(i64, [33]), arr(i64, [55]), arr(i64, [44]), arr(ctypes.c_float, [1.0]),
            arr(p, [A.data_ptr()]), arr(i64, [44]), arr(p, [B.data_ptr()]), arr(i64, [55]),
            arr(ctypes.c_float, [0.0]), arr(p, [C.data_ptr()]), arr(i64, [55]), 0)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        rc = tg.lib.tgemm_batched(*args, torch.cuda.current_stream().cuda_stream)
    assert rc == tg.CAPTURE_UNPLANNED
    # outside capture the same set plans and runs
    assert tg.lib.tgemm_batched(*args, torch.cuda.current_stream().cuda_stream) == 0
    torch.cuda.synchronize()
    ref = oracle.gemm(A.cpu(), B.cpu(), None, 1.0, 0.0)
    assert oracle.normwise_error(C.cpu().numpy(), ref) <= 1e-5


def test_batched_validation(tg):
    A = torch.rand(8, 8, device=DEV)
    with pytest.raises(tg.TgemmError):       # bf16 is not a grouped form
        tg.gemm_batched([A.to(torch.int16)], [A.to(torch.int16)], [A], [1.0], [0.0], "bf16")
    arr = lambda t, v: (t * len(v))(*v)                      # noqa: E731
    i64, p = ctypes.c_int64, ctypes.c_void_p
    bad_ld = tg.lib.tgemm_batched(1, arr(i64, [8]), arr(i64, [8]), arr(i64, [8]),
                                  arr(ctypes.c_float, [1.0]), arr(p, [A.data_ptr()]), arr(i64, [4]),
                                  arr(p, [A.data_ptr()]), arr(i64, [8]), arr(ctypes.c_float, [0.0]),
                                  arr(p, [A.data_ptr()]), arr(i64, [8]), 0, None)
    assert bad_ld == tg.INVALID_VALUE


@pytest.mark.parametrize("dtype", ["f32", "x3"])
def test_autotune_restores_c_and_tuned_plan_is_exact(tg, dtype):
    # The tile-shape tuner times whole-set launches (which overwrite C), puts C back,
    # and later grouped calls use the tuned threshold: still bit-exact on integers.
    rng = np.random.default_rng(53)
    dims = rng.integers(16, 400, size=(40, 3))
    dims[0] = (300, 260, 70)     # 128-tile candidate with edges
    dims[1] = (40, 500, 33)      # 64 tiles under every threshold above 40
    host = _problem_set(dims, 5300, integer=True)
    alphas = [1.0] * len(dims)
    betas = [0.5] * len(dims)
    As = [h[0].to(DEV) for h in host]
    Bs = [h[1].to(DEV) for h in host]
    Cs = [h[2].clone().to(DEV) for h in host]
    before = [c.clone() for c in Cs]
    t = tg.gemm_batched_autotune(As, Bs, Cs, alphas, betas, dtype, reps=2)
    torch.cuda.synchronize()
    print(f"{dtype}: tuned threshold {t}", flush=True)
    assert t["threshold"] in (0, 64, 96, 160, 256, 512, NEVER) and t["large"] in (256, 512, 1024, NEVER)
    assert t["ratio"] == 0 or (t["large"] == NEVER and 0 < t["ratio"] <= 10**6)
    for p, (b, c) in enumerate(zip(before, Cs)):
        assert torch.equal(b, c), f"C of problem {p} not restored"
    tg.gemm_batched(As, Bs, Cs, alphas, betas, dtype)
    torch.cuda.synchronize()
    for p, h in enumerate(host):
        ref = oracle.gemm(h[0], h[1], h[2], alphas[p], betas[p])
        np.testing.assert_array_equal(Cs[p].cpu().numpy().astype(np.float64), ref,
                                      err_msg=f"problem {p} {dims[p]}")


def test_autotune_and_forced_shape_reject_bad_arguments(tg):
    A = torch.ones(8, 8, device=DEV)
    with pytest.raises(tg.TgemmError):
        tg.gemm_batched_autotune([A], [A], [A.clone()], [1.0], [0.0], "f32", reps=0)
    with pytest.raises(tg.TgemmError):
        tg.gemm_batched([A], [A], [A.clone()], [1.0], [0.0], "f32", shape={"threshold": -1, "large": 0})
    for ratio in (-1, 10**6 + 1):
        with pytest.raises(tg.TgemmError):
            tg.gemm_batched([A], [A], [A.clone()], [1.0], [0.0], "f32",
                            shape={"threshold": 0, "large": NEVER, "ratio": ratio})


@pytest.mark.parametrize("ratio", [1, 2000, 3000, 10**6])
@pytest.mark.parametrize("dtype", ["f32", "x3"])
def test_per_problem_rule_is_exact(tg, dtype, ratio):
    # The per-problem rule gives each problem 128 x 128 or 64 x 64 in-place tiles by
    # comparing its tile counts (ratio 1: every problem 128 x 128; 10^6: every problem
    # 64 x 64; 2000 and 3000 split this set between the two).  Bit-exact on integers,
    # C restored between shapes, and the graph replay equals the eager call.
    dims = np.array([(300, 260, 70), (130, 500, 33), (40, 500, 45), (200, 129, 17), (64, 64, 64),
                     (257, 390, 101), (16, 16, 16), (129, 129, 40), (70, 390, 90), (390, 70, 90)])
    # tiles (64, 128): (25, 9), (24, 8), (8, 4), (12, 4), (1, 1), (35, 12), (1, 1), (9, 4),
    # (14, 4), (14, 4): ratio 2000 puts problems 0, 1, 3, 5, 7, 8 and 9 on 128 x 128
    # tiles, ratio 3000 only problems 8 and 9
    host = _problem_set(dims, 5400, integer=True)
    alphas, betas = [1.0] * len(dims), [0.5] * len(dims)
    As = [h[0].to(DEV) for h in host]
    Bs = [h[1].to(DEV) for h in host]
    Cs = [h[2].clone().to(DEV) for h in host]
    shape = {"threshold": NEVER, "large": NEVER, "ratio": ratio}
    tg.gemm_batched(As, Bs, Cs, alphas, betas, dtype, shape=shape)
    torch.cuda.synchronize()
    refs = [oracle.gemm(h[0], h[1], h[2], 1.0, 0.5) for h in host]
    for p in range(len(dims)):
        np.testing.assert_array_equal(Cs[p].cpu().numpy().astype(np.float64), refs[p],
                                      err_msg=f"problem {p} {dims[p]}")
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        tg.gemm_batched(As, Bs, Cs, alphas, betas, dtype, shape=shape)
    for c, h in zip(Cs, host):
        c.copy_(h[2].to(DEV))
    graph.replay()
    torch.cuda.synchronize()
    for p in range(len(dims)):
        np.testing.assert_array_equal(Cs[p].cpu().numpy().astype(np.float64), refs[p],
                                      err_msg=f"replay, problem {p} {dims[p]}")


# small products (M, N <= 16 and <= 32: one wave each) and planned ones
@pytest.mark.parametrize("dims", [(300, 12, 12, 12), (33, 16, 5, 9), (50, 1, 16, 300), (65, 32, 17, 40),
                                  (9, 24, 32, 3), (7, 130, 70, 33), (40, 64, 64, 64), (5, 33, 8, 20)])
@pytest.mark.parametrize("dtype", ["f32", "x3"])
def test_strided_batched_bit_exact(tg, dtype, dims):
    # tgemm_batched_strided: P problems of one shape at fixed strides (here slices of 3-D tensors,
    # C with a row stride wider than N), bit-exact on integers, twice in a row (cached plan)
    P, M, N, K = dims
    g = torch.Generator().manual_seed(sum(dims))
    A = torch.randint(-8, 9, (P, M, K), generator=g).float()
    B = torch.randint(-8, 9, (P, K, N), generator=g).float()
    C0 = torch.randint(-8, 9, (P, M, N), generator=g).float()
    Cbuf = torch.full((P, M, N + 3), float("nan"), device=DEV)
    Cd = Cbuf[:, :, :N]
    Ad, Bd = A.to(DEV), B.to(DEV)
    for rep in range(2):
        Cd.copy_(C0.to(DEV))
        tg.gemm_batched_strided(Ad, Bd, Cd, 1.5, 0.5, dtype)
        torch.cuda.synchronize()
        got = Cd.cpu().numpy().astype(np.float64)
        for p in range(P):
            np.testing.assert_array_equal(got[p], oracle.gemm(A[p], B[p], C0[p], 1.5, 0.5),
                                          err_msg=f"rep {rep} problem {p}")
    assert torch.isnan(Cbuf[:, :, N:]).all()


def test_strided_batched_rejects_overlapping_outputs(tg):
    A = torch.zeros(4, 8, 8, device=DEV)
    C = torch.zeros(64, device=DEV)
    rc = tg.lib.tgemm_batched_strided(4, 8, 8, 8, 1.0, A.data_ptr(), 8, 64, A.data_ptr(), 8, 64, 0.0,
                                      C.data_ptr(), 8, 8, 0, None)
    assert rc == tg.INVALID_VALUE


def test_strided_small_alpha_zero_reads_nothing(tg):
    # small-product path: alpha == 0 gives beta * C with A and B (NaN here) unread
    A = torch.full((10, 12, 12), float("nan"), device=DEV)
    C0 = torch.randint(-8, 9, (10, 12, 12)).float()
    C = C0.to(DEV)
    tg.gemm_batched_strided(A, A, C, 0.0, 0.5)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(C.cpu().numpy(), (0.5 * C0).numpy())
