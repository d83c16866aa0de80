"""tgemm_noalloc (the entry point for callers that cannot allocate) against tgemm.

Both pick the same schedule (the default policy), so their results must agree
bit for bit, except where that schedule is a stream-K form: it needs counters
the library allocates, so tgemm_noalloc runs the same tiles one workgroup per
tile instead, which must then agree bit for bit with that whole-tile schedule.
Both are also held to the oracle's bar.  Two calls in a row, the
second with a smaller problem, check that the shared static workspace keeps no
state a later call depends on; a problem whose packing workspace exceeds the
static array is refused before any launch.
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
    return tgemm


def _ptr(t):
    return t.data_ptr()


def _whole_tile_form(tg, dt, sid):
    """The schedule tgemm_noalloc runs for choice `sid`: itself, or the
    whole-tile schedule of a stream-K form."""
    info = tg.schedule_info(sid)
    if info["split"] == 0:
        return sid
    keys = ("BM", "BN", "BK", "WGM", "WGN", "vec", "lds_bytes", "mfma")
    twin = [s for s, i in tg.schedules(dt) if i["split"] == 0 and all(i[k] == info[k] for k in keys)]
    assert len(twin) == 1
    return twin[0]


def _call(tg, fn, A, B, C, alpha, beta, dt):
    M, K = A.shape
    N = B.shape[1]
    stream = torch.cuda.current_stream().cuda_stream
    return fn(M, N, K, alpha, _ptr(A), A.stride(0), _ptr(B), B.stride(0), beta, _ptr(C), C.stride(0),
              tg.DTYPES[dt], stream)


# (first problem, second smaller problem): both take packed schedules of the rule (f32
# takes them from 2048 tiles of 128 x 256 with M, N > 512, x3 from 768 tiles of 64 x 64 with
# K >= 1024; otherwise in-place tiles, which need no workspace)
SIZES = {"x3": [((2048, 2048, 1024), (2000, 1600, 1100)), ((3000, 2500, 1100), (1700, 1900, 1030))],
         "f32": [((8448, 8192, 640), (8192, 8192, 520)), ((8192, 8448, 600), (8192, 8192, 512))]}


@pytest.mark.parametrize("case", [0, 1])
@pytest.mark.parametrize("dt", ["f32", "x3"])
def test_noalloc_matches_tgemm_two_calls(tg, dt, case):
    for n, (M, N, K) in enumerate(SIZES[dt][case]):
        print(f"noalloc {dt} call {n}: {M}x{N}x{K}", flush=True)
        sid, gm, xcd = tg.select_schedule(M, N, K, dt)
        assert tg.schedule_info(sid)["vec"] == 0, "the case must take a packed schedule"
        A, B, C0 = inputs.gemm_inputs(M, N, K, seed=900 + n)
        Ad, Bd = A.to(DEV), B.to(DEV)
        Cn, Ct, Cw = C0.to(DEV), C0.to(DEV), C0.to(DEV)
        assert _call(tg, tg.lib.tgemm_noalloc, Ad, Bd, Cn, 1.0, 0.5, dt) == 0
        assert _call(tg, tg.lib.tgemm, Ad, Bd, Ct, 1.0, 0.5, dt) == 0
        tg.gemm_with_schedule(Ad, Bd, Cw, 1.0, 0.5, dt, _whole_tile_form(tg, dt, sid), gm, xcd)
        torch.cuda.synchronize()
        assert torch.equal(Cn, Cw)
        if tg.schedule_info(sid)["split"] == 0:
            assert torch.equal(Cn, Ct)
        # the oracle on 48 sampled rows (the f32 problems are too large for it whole)
        rows = torch.from_numpy(np.sort(np.random.default_rng(7 + n).choice(M, 48, replace=False)))
        ref = oracle.gemm(A[rows], B, C0[rows], 1.0, 0.5)
        for out in (Cn, Ct):
            err = oracle.normwise_error(out[rows.to(DEV)].cpu().numpy(), ref)
            assert err <= 1e-5, err


@pytest.mark.parametrize("dt", ["fp8", "bf16"])
def test_noalloc_low_precision_integer_codes(tg, dt):
    # unscaled codes (scale 1) through the packed low-precision path: bit-exact on integers
    for n, (M, N, K) in enumerate([(2048, 1536, 1024), (1536, 2048, 640)]):
        sid, _, _ = tg.select_schedule(M, N, K, dt)
        assert tg.schedule_info(sid)["vec"] == 0, "the case must take a packed schedule"
        A, B, C0 = inputs.integer_inputs(M, N, K, seed=910 + n, r=8)
        if dt == "fp8":
            qa = torch.from_numpy(P.e4m3_encode(A.numpy().astype(np.float64))).to(DEV)
            qb = torch.from_numpy(P.e4m3_encode(B.numpy().astype(np.float64))).to(DEV)
        else:
            qa = torch.from_numpy(P.bf16_bits(A.numpy()).view(np.int16)).to(DEV)
            qb = torch.from_numpy(P.bf16_bits(B.numpy()).view(np.int16)).to(DEV)
        Cn, Ct = C0.to(DEV), C0.to(DEV)
        assert _call(tg, tg.lib.tgemm_noalloc, qa, qb, Cn, 1.5, 0.5, dt) == 0
        assert _call(tg, tg.lib.tgemm, qa, qb, Ct, 1.5, 0.5, dt) == 0
        torch.cuda.synchronize()
        assert torch.equal(Cn, Ct)
        np.testing.assert_array_equal(Cn.cpu().numpy().astype(np.float64), oracle.gemm(A, B, C0, 1.5, 0.5))


def test_noalloc_direct_and_degenerate(tg):
    # a small problem (direct schedule, no workspace) and alpha == 0 (C = beta*C)
    A, B, C0 = inputs.gemm_inputs(100, 70, 50, seed=920)
    Ad, Bd = A.to(DEV), B.to(DEV)
    C = C0.to(DEV)
    assert _call(tg, tg.lib.tgemm_noalloc, Ad, Bd, C, 1.5, 0.5, "f32") == 0
    torch.cuda.synchronize()
    assert oracle.normwise_error(C.cpu().numpy(), oracle.gemm(A, B, C0, 1.5, 0.5)) <= 1e-5
    C = C0.to(DEV)
    assert _call(tg, tg.lib.tgemm_noalloc, Ad, Bd, C, 0.0, 0.5, "x3") == 0
    torch.cuda.synchronize()
    assert torch.equal(C.cpu(), 0.5 * C0)


def test_noalloc_refuses_workspace_beyond_the_array(tg):
    # 8192^3 f32 needs (8192 + 8192) * 8320 * 4 bytes of packing workspace, above 128 MiB:
    # refused before any launch (the pointers are never read)
    f = 0x10000
    rc = tg.lib.tgemm_noalloc(8192, 8192, 8192, 1.0, f, 8192, f, 8192, 0.0, f, 8192, 0, None)
    assert rc == tg.SCRATCH_TOO_SMALL
    assert tg.status_string(rc) == "TGEMM_SCRATCH_TOO_SMALL"
