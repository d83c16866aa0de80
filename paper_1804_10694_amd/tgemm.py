"""Python binding of libtgemm.so (argument marshalling only).

Every entry point has the name of the C function it calls (include/tgemm.h)
without the `tgemm_` prefix.  Tensors are torch tensors on the GPU; the
binding passes their data pointers, row strides and the current HIP stream.
No arithmetic happens here, and there is no CPU fallback: if the library is
not built, importing this module raises.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtgemm.so")

F32, F32_BF16X3, BF16, FP8_E4M3 = 0, 1, 2, 3
DTYPES = {"f32": F32, "x3": F32_BF16X3, "bf16": BF16, "fp8": FP8_E4M3}

SUCCESS, INVALID_VALUE, NOT_SUPPORTED, LAUNCH_FAILED = 0, 1, 2, 3
ALLOC_FAILED, CAPTURE_UNPLANNED, INTERNAL, NO_DEVICE = 4, 5, 6, 7
SCRATCH_TOO_SMALL = 8
NOALLOC_SCRATCH_BYTES = 128 << 20

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run python -m paper_1804_10694_amd.build first")

lib = ctypes.CDLL(LIB_PATH)
_i64, _i32, _f32, _p = ctypes.c_int64, ctypes.c_int, ctypes.c_float, ctypes.c_void_p
_pi64 = ctypes.POINTER(ctypes.c_int64)
_pi32 = ctypes.POINTER(ctypes.c_int32)
_pf32 = ctypes.POINTER(ctypes.c_float)
_pp = ctypes.POINTER(ctypes.c_void_p)

lib.tgemm.argtypes = [_i64, _i64, _i64, _f32, _p, _i64, _p, _i64, _f32, _p, _i64, _i32, _p]
lib.tgemm_noalloc.argtypes = [_i64, _i64, _i64, _f32, _p, _i64, _p, _i64, _f32, _p, _i64, _i32, _p]
lib.tgemm_with_schedule.argtypes = [_i64, _i64, _i64, _f32, _p, _i64, _p, _i64, _f32, _p, _i64,
                                    _i32, _i32, _i32, _i32, _p]
lib.tgemm_scaled.argtypes = [_i64, _i64, _i64, _f32, _p, _i64, _p, _p, _i64, _p, _f32, _p, _i64,
                             _i32, _p]
lib.tgemm_quantize_tiles.argtypes = [_i64, _i64, _p, _i64, _p, _i64, _p, _i32, _p]
lib.tgemm_batched.argtypes = [_i64, _pi64, _pi64, _pi64, _pf32, _pp, _pi64, _pp, _pi64, _pf32, _pp,
                              _pi64, _i32, _p]
lib.tgemm_conv3x3.argtypes = [_i64, _i64, _i64, _i64, _i64, _f32, _p, _p, _f32, _p, _i32, _p]
lib.tgemm_conv3x3_path.argtypes = [_i64, _i64, _i64, _i64, _i64, _f32, _p, _p, _f32, _p, _i32, _i32, _p]
lib.tgemm_conv3x3_packed_shape.argtypes = [_i32, _i32, _p, _p, _p, _p]
lib.tgemm_batched_strided.argtypes = [_i64, _i64, _i64, _i64, _f32, _p, _i64, _i64, _p, _i64, _i64, _f32, _p, _i64,
                                      _i64, _i32, _p]
lib.tgemm_conv2d.argtypes = [_i64, _i64, _i64, _i64, _i64, _i64, _f32, _p, _p, _f32, _p, _i32, _i32, _p]
lib.tgemm_mfma_loop.argtypes = [_i32, _i64, _p, _i64, _p, _p]
lib.tgemm_contract.argtypes = [_i32, _p, _p, _p, _i32, _p, _p, _p, _i32, _p, _p, _p, _f32, _f32, _i32, _p]
lib.tgemm_gemm2.argtypes = [_i64, _i64, _i64, _i64, _f32, _p, _i64, _p, _i64, _i32, _p, _i64, _f32, _p, _i64,
                            _i32, _p]
lib.tgemm_batched_with_shape.argtypes = [_i64, _pi64, _pi64, _pi64, _pf32, _pp, _pi64, _pp, _pi64,
                                         _pf32, _pp, _pi64, _i32, _i32, _i32, _i32, _p]
lib.tgemm_batched_autotune.argtypes = [_i64, _pi64, _pi64, _pi64, _pf32, _pp, _pi64, _pp, _pi64, _pf32,
                                       _pp, _pi64, _i32, _i32, _p, _pi32, _pi32, _pi32]
lib.tgemm_status_string.argtypes = [_i32]
lib.tgemm_status_string.restype = ctypes.c_char_p
lib.tgemm_set_policy.argtypes = [ctypes.c_char_p]
lib.tgemm_schedule_count.argtypes = []
lib.tgemm_schedule_info.argtypes = [_i32, _pi32]
lib.tgemm_tile_map.argtypes = [_i64, _i64, _i32, _i32, _i32, _i32, _pi32, _pi32, _pi32]
lib.tgemm_autotune.argtypes = [_i64, _i64, _i64, _i32, _i32, ctypes.c_char_p]
lib.tgemm_load_tuning_db.argtypes = [ctypes.c_char_p]
lib.tgemm_select_schedule.argtypes = [_i64, _i64, _i64, _i32, _pi32, _pi32, _pi32]
lib.tgemm_mlp_param_count.argtypes = [_i32, _pi32]
lib.tgemm_mlp_param_count.restype = ctypes.c_int64
lib.tgemm_mlp_workspace_count.argtypes = [_i32, _pi32, _i64]
lib.tgemm_mlp_workspace_count.restype = ctypes.c_int64
lib.tgemm_mlp_forward.argtypes = [_i32, _pi32, _p, _i64, _p, _p, _p, _p]
lib.tgemm_mlp_train_step.argtypes = [_i32, _pi32, _p, _p, _p, _p, _i64, _f32, _i64, _p, _p, _p, _p,
                                     _p]
lib.tgemm_adam_step.argtypes = [_i64, _p, _p, _p, _p, _i64, _f32, _p]
lib.tgemm_costmodel_train.argtypes = [ctypes.c_char_p, ctypes.c_char_p, _i32, _i32, _f32,
                                      ctypes.c_uint64, _pf32]
lib.tgemm_costmodel_load.argtypes = [ctypes.c_char_p]
lib.tgemm_costmodel_unload.argtypes = []
lib.tgemm_costmodel_unload.restype = None
lib.tgemm_costmodel_predict.argtypes = [_i64, _i64, _i64, _i32, _pi32, _pi32, _pi32, _pf32]
lib.tgemm_costmodel_predict_all.argtypes = [_i64, _i64, _i64, _i32, _i32, _pi32, _pi32, _pi32,
                                            _pf32]
lib.tgemm_costmodel_select.argtypes = [_i64, _i64, _i64, _i32, _i32, ctypes.c_char_p, _pi32, _pi32,
                                       _pi32, _pi32]
lib.tgemm_costmodel_features.argtypes = [_i64, _i64, _i64, _i32, _i32, _i32, _i32, _pf32]
lib.tgemm_schedule_space_hash.argtypes = []
lib.tgemm_schedule_space_hash.restype = ctypes.c_uint64
lib.tgemm_shutdown.argtypes = []
lib.tgemm_shutdown.restype = None


class TgemmError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {status_string(status)}")


def status_string(status):
    return lib.tgemm_status_string(int(status)).decode()


def _check(rc, where):
    if rc != SUCCESS:
        raise TgemmError(rc, where)
    return rc


def _dtype_code(dtype):
    if isinstance(dtype, str):
        return DTYPES[dtype]
    return int(dtype)


def _stream_handle(stream):
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


_ELEM = {F32: torch.float32, F32_BF16X3: torch.float32, BF16: torch.uint16, FP8_E4M3: torch.uint8}


def _mat(t, name, elem=None):
    """(data_ptr, leading dimension) of a row-major 2-D device tensor."""
    if t is None:
        return None, 1
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dim() != 2:
        raise ValueError(f"{name} must be 2-D")
    if t.shape[1] > 1 and t.stride(1) != 1:
        raise ValueError(f"{name} must have unit column stride (row-major)")
    if elem is not None and t.dtype != elem:
        if not (elem == torch.uint16 and t.dtype in (torch.bfloat16, torch.int16)):
            if not (elem == torch.uint8 and t.dtype in (torch.float8_e4m3fn, torch.int8)):
                raise ValueError(f"{name} has dtype {t.dtype}, expected {elem}")
    ld = t.stride(0) if t.shape[0] > 1 else max(t.shape[1], 1)
    return t.data_ptr(), max(ld, 1)


def gemm(A, B, C, alpha=1.0, beta=0.0, dtype="f32", stream=None):
    """C = alpha*A@B + beta*C in place (tgemm)."""
    dt = _dtype_code(dtype)
    M, K = A.shape
    N = B.shape[1]
    if B.shape[0] != K or tuple(C.shape) != (M, N):
        raise ValueError(f"shape mismatch {tuple(A.shape)} @ {tuple(B.shape)} -> {tuple(C.shape)}")
    pa, lda = _mat(A, "A", _ELEM.get(dt))
    pb, ldb = _mat(B, "B", _ELEM.get(dt))
    pc, ldc = _mat(C, "C", torch.float32)
    _check(lib.tgemm(M, N, K, alpha, pa, lda, pb, ldb, beta, pc, ldc, dt, _stream_handle(stream)),
           "tgemm")
    return C


def gemm_noalloc(A, B, C, alpha=1.0, beta=0.0, dtype="f32", stream=None):
    """C = alpha*A@B + beta*C in place without any device allocation (tgemm_noalloc)."""
    dt = _dtype_code(dtype)
    M, K = A.shape
    N = B.shape[1]
    if B.shape[0] != K or tuple(C.shape) != (M, N):
        raise ValueError(f"shape mismatch {tuple(A.shape)} @ {tuple(B.shape)} -> {tuple(C.shape)}")
    pa, lda = _mat(A, "A", _ELEM.get(dt))
    pb, ldb = _mat(B, "B", _ELEM.get(dt))
    pc, ldc = _mat(C, "C", torch.float32)
    _check(lib.tgemm_noalloc(M, N, K, alpha, pa, lda, pb, ldb, beta, pc, ldc, dt, _stream_handle(stream)),
           "tgemm_noalloc")
    return C


ACT_NONE, ACT_RELU = 0, 1


def gemm2(A, B, D, E, alpha=1.0, beta=0.0, relu=False, dtype="f32", stream=None):
    """E = alpha * act(A@B) @ D + beta*E in place, act = ReLU if relu (tgemm_gemm2): the
    intermediate act(A@B) stays on chip.  Row-major float32 device matrices (unit column stride)."""
    M, K = A.shape
    N1 = B.shape[1]
    N2 = D.shape[1]
    if B.shape[0] != K or D.shape[0] != N1 or tuple(E.shape) != (M, N2):
        raise ValueError(f"shapes do not chain: {tuple(A.shape)} {tuple(B.shape)} {tuple(D.shape)} "
                         f"-> {tuple(E.shape)}")
    pa, lda = _mat(A, "A", torch.float32)
    pb, ldb = _mat(B, "B", torch.float32)
    pd, ldd = _mat(D, "D", torch.float32)
    pe, lde = _mat(E, "E", torch.float32)
    _check(lib.tgemm_gemm2(M, N1, N2, K, alpha, pa, lda, pb, ldb, ACT_RELU if relu else ACT_NONE, pd, ldd,
                           beta, pe, lde, _dtype_code(dtype), _stream_handle(stream)), "tgemm_gemm2")
    return E


def gemm_batched_strided(A, B, C, alpha=1.0, beta=0.0, dtype="f32", stream=None):
    """C[p] = alpha*A[p]@B[p] + beta*C[p] for 3-D float32 device tensors (batch, rows, cols) with
    unit column stride (tgemm_batched_strided)."""
    for name, t in (("A", A), ("B", B), ("C", C)):
        if not t.is_cuda or t.dtype != torch.float32 or t.dim() != 3 or (t.shape[2] > 1 and t.stride(2) != 1):
            raise ValueError(f"{name} must be a 3-D float32 device tensor with unit column stride")
    P, M, K = A.shape
    N = B.shape[2]
    if tuple(B.shape) != (P, K, N) or tuple(C.shape) != (P, M, N):
        raise ValueError("shapes must be A (P, M, K), B (P, K, N), C (P, M, N)")
    ld = lambda t: t.stride(1) if t.shape[1] > 1 else max(t.shape[2], 1)   # noqa: E731
    _check(lib.tgemm_batched_strided(P, M, N, K, alpha, A.data_ptr(), ld(A), A.stride(0), B.data_ptr(), ld(B),
                                     B.stride(0), beta, C.data_ptr(), ld(C), C.stride(0), _dtype_code(dtype),
                                     _stream_handle(stream)), "tgemm_batched_strided")
    return C


def mfma_loop(dtype, iters, sink, stream=None):
    """Launch the matrix-core throughput probe (tgemm_mfma_loop); returns its algorithmic flops.
    `sink` is a float32 device tensor of at least 8192 elements."""
    fl = ctypes.c_double()
    _check(lib.tgemm_mfma_loop(_dtype_code(dtype), iters, sink.data_ptr(), sink.numel(), ctypes.byref(fl),
                               _stream_handle(stream)), "tgemm_mfma_loop")
    return fl.value


def contract(A, modes_a, B, modes_b, C, modes_c, alpha=1.0, beta=0.0, dtype="f32", stream=None):
    """C[modes_c] = alpha * sum A[modes_a] * B[modes_b] + beta * C (tgemm_contract): contiguous
    float32 device tensors, modes given as sequences of integer labels."""
    def arrs(t, modes, name):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous float32 device tensor")
        if len(modes) != t.dim():
            raise ValueError(f"{name} has {t.dim()} modes, {len(modes)} labels given")
        m = (ctypes.c_int32 * max(len(modes), 1))(*modes)
        e = (ctypes.c_int64 * max(t.dim(), 1))(*t.shape)
        return len(modes), m, e, t.data_ptr()
    na, ma, ea, pa = arrs(A, modes_a, "A")
    nb, mb, eb, pb = arrs(B, modes_b, "B")
    nc, mc, ec, pc = arrs(C, modes_c, "C")
    _check(lib.tgemm_contract(na, ma, ea, pa, nb, mb, eb, pb, nc, mc, ec, pc, alpha, beta, _dtype_code(dtype),
                              _stream_handle(stream)), "tgemm_contract")
    return C


def gemm_raw(M, N, K, alpha, pa, lda, pb, ldb, beta, pc, ldc, dtype, stream=None):
    """tgemm on raw device pointers; returns the status code (no exception)."""
    return lib.tgemm(M, N, K, alpha, pa, lda, pb, ldb, beta, pc, ldc, _dtype_code(dtype),
                     _stream_handle(stream) if stream is not False else None)


def gemm_with_schedule(A, B, C, alpha, beta, dtype, schedule_id, group_m=8, xcd_remap=1,
                       stream=None):
    dt = _dtype_code(dtype)
    M, K = A.shape
    N = B.shape[1]
    pa, lda = _mat(A, "A", _ELEM.get(dt))
    pb, ldb = _mat(B, "B", _ELEM.get(dt))
    pc, ldc = _mat(C, "C", torch.float32)
    _check(lib.tgemm_with_schedule(M, N, K, alpha, pa, lda, pb, ldb, beta, pc, ldc, dt,
                                   schedule_id, group_m, xcd_remap, _stream_handle(stream)),
           "tgemm_with_schedule")
    return C


def gemm_scaled(A, sA, B, sB, C, alpha=1.0, beta=0.0, dtype="fp8", stream=None):
    dt = _dtype_code(dtype)
    M, K = A.shape
    N = B.shape[1]
    pa, lda = _mat(A, "A", _ELEM.get(dt))
    pb, ldb = _mat(B, "B", _ELEM.get(dt))
    pc, ldc = _mat(C, "C", torch.float32)
    _check(lib.tgemm_scaled(M, N, K, alpha, pa, lda, sA.data_ptr(), pb, ldb, sB.data_ptr(), beta,
                            pc, ldc, dt, _stream_handle(stream)), "tgemm_scaled")
    return C


def quantize_tiles(X, dtype="fp8", stream=None):
    """(Q, S): per-128x128-tile quantised X and its scale grid (tgemm_quantize_tiles)."""
    dt = _dtype_code(dtype)
    rows, cols = X.shape
    px, ldx = _mat(X, "X", torch.float32)
    qdt = torch.uint8 if dt == FP8_E4M3 else torch.int16   # bf16 bit patterns
    Q = torch.empty(rows, cols, dtype=qdt, device=X.device)
    S = torch.empty(-(-rows // 128), -(-cols // 128), dtype=torch.float32, device=X.device)
    _check(lib.tgemm_quantize_tiles(rows, cols, px, ldx, Q.data_ptr(), max(cols, 1), S.data_ptr(),
                                    dt, _stream_handle(stream)), "tgemm_quantize_tiles")
    return Q, S


def _arr(ctype, values):
    return (ctype * len(values))(*values)


def gemm_batched(As, Bs, Cs, alphas, betas, dtype="f32", stream=None, shape=None):
    """Grouped gemm over lists of tensors (tgemm_batched): C_p = a_p A_p B_p + b_p C_p.
    shape: None (tuned or default plan shape) or {"threshold": T, "large": L}
    with an optional "ratio" (per-problem rule, per mille; tgemm_batched_with_shape)."""
    args = _batched_args(As, Bs, Cs, alphas, betas, dtype)
    if shape is None:
        _check(lib.tgemm_batched(*args, _stream_handle(stream)), "tgemm_batched")
    else:
        _check(lib.tgemm_batched_with_shape(*args, int(shape["threshold"]), int(shape["large"]),
                                            int(shape.get("ratio", 0)), _stream_handle(stream)),
               "tgemm_batched_with_shape")


def _batched_args(As, Bs, Cs, alphas, betas, dtype):
    dt = _dtype_code(dtype)
    n = len(As)
    Ms, Ns, Ks, pa, pb, pc, la, lb, lc = [], [], [], [], [], [], [], [], []
    for A, B, C in zip(As, Bs, Cs):
        M, K = A.shape
        N = B.shape[1]
        a, lda = _mat(A, "A", _ELEM.get(dt))
        b, ldb = _mat(B, "B", _ELEM.get(dt))
        c, ldc = _mat(C, "C", torch.float32)
        Ms.append(M); Ns.append(N); Ks.append(K)
        pa.append(a); pb.append(b); pc.append(c)
        la.append(lda); lb.append(ldb); lc.append(ldc)
    return (n, _arr(_i64, Ms), _arr(_i64, Ns), _arr(_i64, Ks), _arr(_f32, list(alphas)),
            _arr(_p, pa), _arr(_i64, la), _arr(_p, pb), _arr(_i64, lb), _arr(_f32, list(betas)),
            _arr(_p, pc), _arr(_i64, lc), dt)


def gemm_batched_autotune(As, Bs, Cs, alphas, betas, dtype="f32", reps=5, stream=None):
    """Plan-shape tuning of a grouped set (tgemm_batched_autotune); returns
    {"threshold": T, "large": L, "ratio": R} (2**31 - 1: never; R = 0: the
    threshold rule, else the per-problem rule at cost ratio R / 1000)."""
    args = _batched_args(As, Bs, Cs, alphas, betas, dtype)
    thr, large, ratio = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib.tgemm_batched_autotune(*args, reps, _stream_handle(stream), ctypes.byref(thr),
                                      ctypes.byref(large), ctypes.byref(ratio)), "tgemm_batched_autotune")
    return {"threshold": thr.value, "large": large.value, "ratio": ratio.value}


CONV_AUTO, CONV_DIRECT, CONV_PACKED = 0, 1, 2


def conv3x3_packed_shapes(dtype="f32"):
    """(bm, bn, bk, stages) of each packed conv tile shape of `dtype`
    (tgemm_conv3x3_packed_shape)."""
    out = []
    while True:
        v = [ctypes.c_int32() for _ in range(4)]
        if lib.tgemm_conv3x3_packed_shape(_dtype_code(dtype), len(out), *[ctypes.byref(x) for x in v]) != 0:
            return out
        out.append(tuple(x.value for x in v))


CONV_RUNTIME_R = 0x100


def conv2d(X, Wt, Y, alpha=1.0, beta=0.0, dtype="f32", stream=None, path="auto", shape=0, runtime_r=False):
    """R x R same-padding convolution as an implicit gemm (tgemm_conv2d), R = Wt.shape[0] odd:
    Y = alpha * conv(X, Wt) + beta * Y, with X (batch, H, W, Cin), Wt (R, R, Cin, Cout) and
    Y (batch, H, W, Cout) contiguous float32 device tensors.  path "auto" (the library's
    choice), "direct", or "packed" with tile shape index `shape`; runtime_r selects the
    kernel that takes R at run time also for 3 x 3."""
    import torch
    for name, t in (("X", X), ("Wt", Wt), ("Y", Y)):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 \
                or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous float32 device tensor")
    nb, H, W, cin = X.shape
    R = Wt.shape[0]
    if tuple(Wt.shape[:3]) != (R, R, cin) or tuple(Y.shape) != (nb, H, W, Wt.shape[3]):
        raise ValueError("shapes must be X (b, H, W, Cin), Wt (R, R, Cin, Cout), Y (b, H, W, Cout)")
    if path == "auto":
        code = CONV_AUTO
    elif path == "direct":
        code = CONV_DIRECT
    elif path == "packed":
        code = CONV_PACKED + int(shape)
    else:
        raise ValueError(f"unknown conv path {path!r}")
    if runtime_r:
        code |= CONV_RUNTIME_R
    _check(lib.tgemm_conv2d(nb, H, W, cin, Wt.shape[3], R, alpha, X.data_ptr(), Wt.data_ptr(), beta,
                            Y.data_ptr(), _dtype_code(dtype), code, _stream_handle(stream)), "tgemm_conv2d")


def conv3x3(X, Wt, Y, alpha=1.0, beta=0.0, dtype="f32", stream=None, path="auto", shape=0):
    """3x3 same-padding convolution as an implicit gemm (tgemm_conv3x3_path): conv2d with a
    3 x 3 x Cin x Cout filter."""
    if Wt.dim() != 4 or tuple(Wt.shape[:2]) != (3, 3):
        raise ValueError("conv3x3 takes a (3, 3, Cin, Cout) filter")
    conv2d(X, Wt, Y, alpha, beta, dtype, stream, path, shape)


def set_policy(policy):
    _check(lib.tgemm_set_policy(policy.encode()), "tgemm_set_policy")


def schedule_count():
    return lib.tgemm_schedule_count()


def schedule_info(sid):
    buf = (ctypes.c_int32 * 11)()
    _check(lib.tgemm_schedule_info(sid, buf), "tgemm_schedule_info")
    keys = ("dtype", "BM", "BN", "BK", "WGM", "WGN", "vec", "lds_bytes", "split", "mfma", "inplace")
    return dict(zip(keys, list(buf)))


def schedules(dtype=None):
    out = []
    for i in range(schedule_count()):
        info = schedule_info(i)
        if dtype is None or info["dtype"] == _dtype_code(dtype):
            out.append((i, info))
    return out


def schedule_key(sid):
    """Readable, unique name of a compiled schedule: dtype, tile sizes, wave grid, load
    width (vec0: packed operands) and LDS bytes (which tell the pipeline depths apart)."""
    i = schedule_info(sid)
    return (f"sched:{i['dtype']}:{i['BM']}x{i['BN']}x{i['BK']}:{i['WGM']}x{i['WGN']}:"
            f"vec{i['vec']}:lds{i['lds_bytes']}" + (":streamk" if i["split"] else "")
            + (":mfma16" if i["mfma"] == 16 else "") + (":inplace" if i["inplace"] else ""))


def tile_map(M, N, BM, BN, group_m, xcd_remap):
    T = (-(-M // BM)) * (-(-N // BN))
    tm = (ctypes.c_int32 * T)()
    tn = (ctypes.c_int32 * T)()
    fl = (ctypes.c_int32 * T)()
    _check(lib.tgemm_tile_map(M, N, BM, BN, group_m, xcd_remap, tm, tn, fl), "tgemm_tile_map")
    return list(tm), list(tn), list(fl)


def autotune(M, N, K, dtype, reps, db_path):
    best = lib.tgemm_autotune(M, N, K, _dtype_code(dtype), reps, db_path.encode())
    if best < 0:
        raise TgemmError(-best, "tgemm_autotune")
    return best


def load_tuning_db(path):
    n = lib.tgemm_load_tuning_db(path.encode())
    if n < 0:
        raise TgemmError(-n, "tgemm_load_tuning_db")
    return n


def select_schedule(M, N, K, dtype):
    sid, gm, xcd = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib.tgemm_select_schedule(M, N, K, _dtype_code(dtype), ctypes.byref(sid),
                                     ctypes.byref(gm), ctypes.byref(xcd)), "tgemm_select_schedule")
    return sid.value, gm.value, xcd.value


def schedule_space_hash():
    return int(lib.tgemm_schedule_space_hash())


def _dims(dims):
    return (ctypes.c_int32 * len(dims))(*dims), len(dims) - 1


def mlp_param_count(dims):
    d, layers = _dims(dims)
    n = lib.tgemm_mlp_param_count(layers, d)
    if n < 0:
        raise TgemmError(-n, "tgemm_mlp_param_count")
    return n


def mlp_workspace(dims, rows, device="cuda"):
    d, layers = _dims(dims)
    n = lib.tgemm_mlp_workspace_count(layers, d, rows)
    if n < 0:
        raise TgemmError(-n, "tgemm_mlp_workspace_count")
    return torch.empty(n, dtype=torch.float32, device=device)


def mlp_forward(dims, params, X, out=None, work=None, stream=None):
    d, layers = _dims(dims)
    rows = X.shape[0]
    if out is None:
        out = torch.empty(rows, dtype=torch.float32, device=X.device)
    if work is None:
        work = mlp_workspace(dims, rows, X.device)
    _check(lib.tgemm_mlp_forward(layers, d, params.data_ptr(), rows, X.data_ptr(), out.data_ptr(),
                                 work.data_ptr(), _stream_handle(stream)), "tgemm_mlp_forward")
    return out


def mlp_train_step(dims, params, grads, m, v, step, lr, X, y, loss, work, stream=None):
    d, layers = _dims(dims)
    _check(lib.tgemm_mlp_train_step(layers, d, params.data_ptr(), grads.data_ptr(), m.data_ptr(),
                                    v.data_ptr(), step, lr, X.shape[0], X.data_ptr(), y.data_ptr(),
                                    loss.data_ptr(), work.data_ptr(), _stream_handle(stream)),
           "tgemm_mlp_train_step")


def adam_step(params, grads, m, v, step, lr, stream=None):
    _check(lib.tgemm_adam_step(params.numel(), params.data_ptr(), grads.data_ptr(), m.data_ptr(),
                               v.data_ptr(), step, lr, _stream_handle(stream)), "tgemm_adam_step")


def costmodel_train(db_path, weights_out, epochs=60, batch=512, lr=1e-3, seed=5):
    loss = ctypes.c_float()
    _check(lib.tgemm_costmodel_train(db_path.encode(), weights_out.encode(), epochs, batch, lr, seed,
                                     ctypes.byref(loss)), "tgemm_costmodel_train")
    return loss.value


def costmodel_load(path):
    _check(lib.tgemm_costmodel_load(path.encode()), "tgemm_costmodel_load")


def costmodel_unload():
    lib.tgemm_costmodel_unload()


def costmodel_predict(M, N, K, dtype):
    """(schedule, group_m, xcd, predicted_ms) or None when the model cannot answer."""
    sid, gm, xcd, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_float()
    rc = lib.tgemm_costmodel_predict(M, N, K, _dtype_code(dtype), ctypes.byref(sid), ctypes.byref(gm),
                                     ctypes.byref(xcd), ctypes.byref(ms))
    if rc == NOT_SUPPORTED:
        return None
    _check(rc, "tgemm_costmodel_predict")
    return sid.value, gm.value, xcd.value, ms.value


def costmodel_predict_all(M, N, K, dtype, max_rows=4096):
    sid = (ctypes.c_int32 * max_rows)()
    gm = (ctypes.c_int32 * max_rows)()
    xcd = (ctypes.c_int32 * max_rows)()
    ms = (ctypes.c_float * max_rows)()
    n = lib.tgemm_costmodel_predict_all(M, N, K, _dtype_code(dtype), max_rows, sid, gm, xcd, ms)
    if n < 0:
        raise TgemmError(-n, "tgemm_costmodel_predict_all")
    return [(sid[i], gm[i], xcd[i], ms[i]) for i in range(n)]


def costmodel_select(M, N, K, dtype, reps, db_path):
    sid, gm, xcd, fb = (ctypes.c_int32() for _ in range(4))
    _check(lib.tgemm_costmodel_select(M, N, K, _dtype_code(dtype), reps, db_path.encode(),
                                      ctypes.byref(sid), ctypes.byref(gm), ctypes.byref(xcd),
                                      ctypes.byref(fb)), "tgemm_costmodel_select")
    return sid.value, gm.value, xcd.value, bool(fb.value)


def costmodel_features(M, N, K, dtype, sid, group_m, xcd):
    out = (ctypes.c_float * 22)()
    _check(lib.tgemm_costmodel_features(M, N, K, _dtype_code(dtype), sid, group_m, xcd, out),
           "tgemm_costmodel_features")
    return list(out)


def shutdown():
    lib.tgemm_shutdown()
