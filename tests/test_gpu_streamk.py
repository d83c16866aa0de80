"""GPU parity of the stream-K forms of the packed schedules against the FP64 oracle.

A stream-K launch splits the (tile, K panel) iterations of C = alpha*A*B + beta*C
(Tiramisu paper, Section I) evenly over one resident wave of workgroups; a tile
shared by several workgroups is summed in K order by the last one to finish.
Bars: bit-exact on small-integer inputs (every partial sum is an integer below
2^24, so the split changes nothing); normwise error <= 1e-5 on U[-1, 1] inputs;
bitwise-equal repeats and graph replays (the summation order does not depend
on which workgroup finishes last, and the per-tile counters are left at zero).
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import precision as P
from paper_1804_10694_amd import inputs

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def tg():
    from paper_1804_10694_amd import tgemm
    tgemm.set_policy("default")
    yield tgemm
    tgemm.set_policy("default")


def _sk(tg, dtype):
    return [(sid, info) for sid, info in tg.schedules(dtype) if info["split"] == 1]


def _codes(X, dtype):
    if dtype == "fp8":
        return torch.from_numpy(P.e4m3_encode(X.numpy().astype(np.float64)))
    return torch.from_numpy(P.bf16_bits(X.numpy()).view(np.int16))


def test_every_dtype_has_stream_k_forms(tg):
    for dt in ("f32", "x3", "bf16", "fp8"):
        sk = _sk(tg, dt)
        assert sk, dt
        for sid, info in sk:
            assert info["vec"] == 0
            twin = [s for s, i in tg.schedules(dt) if i["split"] == 0 and
                    all(i[k] == info[k] for k in ("BM", "BN", "BK", "WGM", "WGN", "vec", "lds_bytes", "mfma"))]
            assert len(twin) == 1, tg.schedule_key(sid)


# Shapes: a few tiles split over many workgroups (every range a piece of a tile),
# ragged in every dimension, and one whose tiles are each shared by two or three.
SHAPES = [(300, 208, 272), (1000, 777, 1029), (2100, 1500, 1153)]


@pytest.mark.parametrize("dtype", ["f32", "x3"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_stream_k_bit_exact_on_integers(tg, dtype, shape):
    M, N, K = shape
    A, B, C0 = inputs.integer_inputs(M, N, K, seed=60)
    Ad, Bd = A.to(DEV), B.to(DEV)
    for alpha, beta in [(1.5, 0.5), (1.0, 0.0)]:
        ref = oracle.gemm(A, B, C0, alpha, beta)
        for sid, info in _sk(tg, dtype):
            for gm in (8, 1):
                print(f"stream-K {tg.schedule_key(sid)} {shape} alpha={alpha} beta={beta} gm={gm}",
                      flush=True)
                C = C0.to(DEV)
                if beta == 0.0:
                    C.fill_(float("nan"))   # beta == 0: C is written, never read
                tg.gemm_with_schedule(Ad, Bd, C, alpha, beta, dtype, sid, gm, 1)
                torch.cuda.synchronize()
                np.testing.assert_array_equal(C.cpu().numpy().astype(np.float64), ref,
                                              err_msg=tg.schedule_key(sid))


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_stream_k_low_precision_codes_exact(tg, dtype):
    for shape in SHAPES[:2]:
        M, N, K = shape
        A, B, C0 = inputs.integer_inputs(M, N, K, seed=61, r=8)
        ref = oracle.gemm(A, B, C0, 1.5, 0.5)
        qa, qb = _codes(A, dtype).to(DEV), _codes(B, dtype).to(DEV)
        for sid, info in _sk(tg, dtype):
            print(f"stream-K {tg.schedule_key(sid)} {shape}", flush=True)
            C = C0.to(DEV)
            tg.gemm_with_schedule(qa, qb, C, 1.5, 0.5, dtype, sid)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(C.cpu().numpy().astype(np.float64), ref)


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_stream_k_scaled_against_dequantised_product(tg, dtype):
    # per-tile scales that change along K: each range's partial is rescaled to its last
    # K block before the ranges are summed
    M, N, K = 700, 600, 1100
    A, B = inputs.lowprec_inputs(M, N, K, seed=62)
    quant = P.quantize_tiles_e4m3 if dtype == "fp8" else P.quantize_tiles_bf16
    QA, SA = quant(A.numpy())
    QB, SB = quant(B.numpy())
    Ad = P.dequantize_tiles(P.decode(QA, dtype), SA, 128)
    Bd = P.dequantize_tiles(P.decode(QB, dtype), SB, 128)
    ref = oracle.gemm(Ad, Bd, None, 1.0, 0.0)
    view = np.uint8 if dtype == "fp8" else np.int16
    qa = torch.from_numpy(QA.view(view)).to(DEV)
    qb = torch.from_numpy(QB.view(view)).to(DEV)
    sa, sb = torch.from_numpy(SA).to(DEV), torch.from_numpy(SB).to(DEV)
    bar = 2.0 ** -12 if dtype == "fp8" else 1e-5
    for sid, info in _sk(tg, dtype):
        tg.set_policy(f"force:{sid}")
        C = torch.full((M, N), float("nan"), device=DEV)
        tg.gemm_scaled(qa, sa, qb, sb, C, 1.0, 0.0, dtype)
        torch.cuda.synchronize()
        err = oracle.normwise_error(C.cpu().numpy(), ref)
        print(f"stream-K scaled {tg.schedule_key(sid)} error {err:.3e}", flush=True)
        assert err <= bar, (tg.schedule_key(sid), err)
    tg.set_policy("default")


@pytest.mark.parametrize("dtype", ["f32", "x3"])
def test_stream_k_normwise_error_and_repeats(tg, dtype):
    M, N, K = 1500, 1200, 2053
    A, B, C0 = inputs.gemm_inputs(M, N, K, seed=63)
    ref = oracle.gemm(A, B, C0, 1.0, 1.0)
    Ad, Bd = A.to(DEV), B.to(DEV)
    for sid, info in _sk(tg, dtype):
        outs = []
        for rep in range(3):
            C = C0.to(DEV)
            tg.gemm_with_schedule(Ad, Bd, C, 1.0, 1.0, dtype, sid)
            torch.cuda.synchronize()
            outs.append(C.cpu())
        err = oracle.normwise_error(outs[0].numpy(), ref)
        print(f"stream-K {tg.schedule_key(sid)} error {err:.3e}", flush=True)
        assert err <= 1e-5
        for o in outs[1:]:
            assert torch.equal(o, outs[0]), "stream-K repeats differ"


def test_stream_k_graph_replay_matches_eager(tg):
    M, N, K = 1000, 777, 1029
    A, B, C0 = inputs.gemm_inputs(M, N, K, seed=64)
    Ad, Bd = A.to(DEV), B.to(DEV)
    for dtype in ("f32", "x3"):
        sid = _sk(tg, dtype)[0][0]
        C = C0.to(DEV)
        tg.gemm_with_schedule(Ad, Bd, C, 1.0, 0.5, dtype, sid)   # allocates the workspace
        torch.cuda.synchronize()
        eager = C.clone()
        s = torch.cuda.Stream()
        Cg = C0.to(DEV)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s):
            tg.gemm_with_schedule(Ad, Bd, Cg, 1.0, 0.5, dtype, sid, stream=s)  # workspace of s
            torch.cuda.synchronize()
            with torch.cuda.graph(g, stream=s):
                tg.gemm_with_schedule(Ad, Bd, Cg, 1.0, 0.5, dtype, sid, stream=s)
        for rep in range(3):
            Cg.copy_(C0.to(DEV))
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(Cg, eager), f"{dtype} replay {rep} differs from eager"
            Ce = C0.to(DEV)   # eager work between replays
            tg.gemm_with_schedule(Ad, Bd, Ce, 1.0, 0.5, dtype, sid)
            torch.cuda.synchronize()
            assert torch.equal(Ce, eager)
