"""Precision forms of the gemm library, written out from their definitions.

Test infrastructure only (see the package docstring).

The Tiramisu paper computes gemm in single precision (Section VI-A, sgemm);
the forms below are project additions, so each function states the reading it
implements:

  bf16_rne(x)          round float32 to bfloat16 (8 significant bits, the
                       float32 exponent range), round-to-nearest-even.
  split_bf16x3(a)      hi = RNE_bf16(a), lo = RNE_bf16(a - hi).  a - hi is
                       exact in float32, so it is formed in float32.
  gemm_x3_expected     alpha * sum_k (hiA hiB + hiA loB + loA hiB) + beta*C0
                       in FP64: the split product with the lo*lo term dropped.
  e4m3_rne_sat(x)      round to the OCP E4M3FN grid (4 exponent bits, bias 7,
                       3 mantissa bits, subnormals, largest finite 448, no
                       infinities), nearest-even, values beyond 448 saturate.
  quantize_tiles_*     one FP32 scale per 128 x 128 tile of a row-major matrix
                       (the last tiles may be partial):
                         e4m3: s = the power of two with amax / s in
                               (224, 448] (exponent clamped to the float32
                               normal range), s = 1 when amax = 0,
                               q = e4m3_rne_sat(x / s) (exact division);
                         bf16: s = 2^ceil(log2 amax), s = 1 when amax = 0,
                               q = RNE_bf16(x / s) (exact power-of-two scale).
  dequantize_tiles     q * s in FP64 (exact: at most 8 + 24 significant bits).

Every decision that turns a float into a code is taken in float32, the
precision the GPU quantiser uses, so the codes can be compared bit for bit.
"""
import numpy as np

from .gemm import gemm

TILE = 128
E4M3_MAX = 448.0


# --------------------------------------------------------------------- bf16
def bf16_rne(x):
    """Round float32 values to the nearest bfloat16 value, ties to even.

    A bfloat16 value is a float32 whose low 16 bits are zero.  For a finite
    float32 with bit pattern u the two candidates are the truncation
    (u >> 16) << 16 and the next value away from zero ((u >> 16) + 1) << 16;
    the dropped 16 bits decide: above half -> up, below half -> down, exactly
    half -> whichever of the two has an even upper half.  A carry out of the
    mantissa moves to the next binade (or to infinity), as IEEE rounding does.
    NaN stays NaN.
    """
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = x.view(np.uint32).astype(np.uint64)
    upper = u >> np.uint64(16)
    lower = u & np.uint64(0xFFFF)
    half = np.uint64(0x8000)
    up = (lower > half) | ((lower == half) & ((upper & np.uint64(1)) == 1))
    upper = upper + up.astype(np.uint64)
    out = (upper << np.uint64(16)).astype(np.uint32).view(np.float32)
    return np.where(np.isnan(x), np.float32(np.nan), out).astype(np.float32)


def bf16_bits(x_bf16_valued):
    """The 16-bit pattern of float32 values that are already bf16 values."""
    x = np.ascontiguousarray(np.asarray(x_bf16_valued, dtype=np.float32))
    return (x.view(np.uint32) >> np.uint32(16)).astype(np.uint16)


def bf16_from_bits(bits):
    b = np.asarray(bits, dtype=np.uint16).astype(np.uint32) << np.uint32(16)
    return b.view(np.float32)


def split_bf16x3(a):
    """(hi, lo) with hi = RNE_bf16(a) and lo = RNE_bf16(a - hi), as float32."""
    a = np.asarray(a, dtype=np.float32)
    hi = bf16_rne(a)
    r = (a - hi).astype(np.float32)  # exact: a and hi share the leading bits
    lo = bf16_rne(r)
    return hi, lo


def gemm_x3_expected(A, B, C0, alpha, beta):
    """FP64 alpha*(hiA@hiB + hiA@loB + loA@hiB) + beta*C0."""
    A = np.asarray(A, dtype=np.float32)
    B = np.asarray(B, dtype=np.float32)
    hA, lA = split_bf16x3(A)
    hB, lB = split_bf16x3(B)
    s = gemm(hA, hB) + gemm(hA, lB) + gemm(lA, hB)
    out = alpha * s
    if beta != 0.0:
        out = out + beta * np.asarray(C0, dtype=np.float64)
    return out


# --------------------------------------------------------------------- e4m3
def e4m3_rne_sat(x):
    """Nearest E4M3FN value (ties to even), saturating at +-448; float64 out.

    For |x| >= 2^-6 (normal range) write |x| = m * 2^e with 1 <= m < 2; the
    grid spacing there is 2^(e-3).  Below 2^-6 the spacing is the subnormal
    step 2^-9.  |x| / spacing is exact in FP64; rint() rounds it half to even,
    which picks the even mantissa on a tie.
    """
    x = np.asarray(x, dtype=np.float64)
    ax = np.abs(x)
    frac, p = np.frexp(ax)            # ax = frac * 2^p, 0.5 <= frac < 1
    e = p.astype(np.int64) - 1        # ax = (2 frac) * 2^e
    e = np.maximum(e, -6)             # subnormals share the 2^-6 binade step
    step = np.ldexp(1.0, (e - 3).astype(np.int64))
    q = np.rint(ax / step) * step
    q = np.minimum(q, E4M3_MAX)
    q = np.where(ax >= E4M3_MAX, E4M3_MAX, q)
    out = np.copysign(q, x)
    return np.where(np.isnan(x), np.nan, out)


def e4m3_encode(v):
    """Byte code of E4M3FN values (float64 inputs already on the grid)."""
    v = np.asarray(v, dtype=np.float64)
    sign = (np.signbit(v)).astype(np.uint8) << np.uint8(7)
    av = np.abs(v)
    frac, p = np.frexp(av)
    e = p.astype(np.int64) - 1
    normal = av >= 2.0 ** -6
    exp_field = np.where(normal, e + 7, 0)
    mant = np.where(normal, av / np.ldexp(1.0, e) * 8.0 - 8.0, av / 2.0 ** -9)
    code = (exp_field.astype(np.int64) << 3) | np.rint(mant).astype(np.int64)
    code = np.where(av == 0.0, 0, code)
    code = np.where(np.isnan(v), 0x7F, code).astype(np.uint8)
    return code | sign


def e4m3_decode(code):
    """float64 values of E4M3FN byte codes (0x7F/0xFF decode to NaN)."""
    c = np.asarray(code, dtype=np.uint8).astype(np.int64)
    sign = np.where(c & 0x80, -1.0, 1.0)
    ef = (c >> 3) & 0xF
    m = c & 0x7
    val = np.where(ef == 0, m * 2.0 ** -9,
                   (1.0 + m / 8.0) * np.ldexp(1.0, (ef - 7).astype(np.int64)))
    val = np.where((ef == 0xF) & (m == 0x7), np.nan, val)
    return sign * val


# ------------------------------------------------------------ tile scaling
def _tiles(rows, cols, tile=TILE):
    for ti in range(0, rows, tile):
        for tj in range(0, cols, tile):
            yield ti // tile, tj // tile, slice(ti, min(ti + tile, rows)), \
                slice(tj, min(tj + tile, cols))


def scale_grid_shape(rows, cols, tile=TILE):
    return (-(-rows // tile), -(-cols // tile))


def quantize_tiles_e4m3(X, tile=TILE):
    """(codes uint8 [rows, cols], scales float32 [ceil(rows/t), ceil(cols/t)])."""
    X = np.asarray(X, dtype=np.float32)
    rows, cols = X.shape
    S = np.ones(scale_grid_shape(rows, cols, tile), dtype=np.float32)
    Q = np.zeros((rows, cols), dtype=np.uint8)
    for bi, bj, rs, cs in _tiles(rows, cols, tile):
        blk = X[rs, cs]
        amax = np.float32(np.max(np.abs(blk))) if blk.size else np.float32(0)
        s = np.float32(1.0)
        if amax > 0:
            # amax = f 2^p with 0.5 <= f < 1, and 448 = 0.875 * 2^9: the smallest e
            # with 448 * 2^e >= amax is p - 9 when f <= 0.875, else p - 8
            f, p = np.frexp(amax)
            e = int(p) - 9 if f <= 0.875 else int(p) - 8
            s = np.float32(np.ldexp(1.0, min(max(e, -126), 127)))
        S[bi, bj] = s
        y = (blk / s).astype(np.float32)          # exact: s is a power of two
        Q[rs, cs] = e4m3_encode(e4m3_rne_sat(y))
    return Q, S


def quantize_tiles_bf16(X, tile=TILE):
    """(bf16 bit patterns uint16 [rows, cols], power-of-two scales float32)."""
    X = np.asarray(X, dtype=np.float32)
    rows, cols = X.shape
    S = np.ones(scale_grid_shape(rows, cols, tile), dtype=np.float32)
    Q = np.zeros((rows, cols), dtype=np.uint16)
    for bi, bj, rs, cs in _tiles(rows, cols, tile):
        blk = X[rs, cs]
        amax = float(np.max(np.abs(blk))) if blk.size else 0.0
        if amax > 0:
            frac, p = np.frexp(amax)      # amax = frac * 2^p, 0.5 <= frac < 1
            e = p - 1 if frac == 0.5 else p  # ceil(log2(amax))
            s = np.float32(np.ldexp(1.0, int(e)))
        else:
            s = np.float32(1.0)
        S[bi, bj] = s
        Q[rs, cs] = bf16_bits(bf16_rne((blk / s).astype(np.float32)))
    return Q, S


def dequantize_tiles(values, S, tile=TILE):
    """FP64 q * s for decoded values [rows, cols] and their scale grid."""
    V = np.asarray(values, dtype=np.float64)
    rows, cols = V.shape
    out = np.empty_like(V)
    for bi, bj, rs, cs in _tiles(rows, cols, tile):
        out[rs, cs] = V[rs, cs] * np.float64(S[bi, bj])
    return out


def dequantize_e4m3(Q, S, tile=TILE):
    return dequantize_tiles(e4m3_decode(Q), S, tile)


def dequantize_bf16(Q, S, tile=TILE):
    return dequantize_tiles(bf16_from_bits(Q).astype(np.float64), S, tile)


# ----------------------------------------------------------- scaled gemm
def decode(Q, dtype):
    """float64 values of codes: dtype 'fp8' (E4M3FN bytes) or 'bf16' (16-bit patterns)."""
    if dtype == "fp8":
        return e4m3_decode(Q)
    return bf16_from_bits(Q).astype(np.float64)


def gemm_scaled_expected(QA, SA, QB, SB, C0, alpha, beta, dtype, tile=TILE):
    """FP64 alpha * dequant(QA, SA) @ dequant(QB, SB) + beta * C0.

    In exact arithmetic this equals the per-tile form
    alpha * sum_kb SA[i/t, kb] SB[kb, j/t] sum_{k in kb} qA[i,k] qB[k,j] + beta*C0,
    because every product qA*qB inside K block kb carries the same two scales.
    """
    Ad = dequantize_tiles(decode(QA, dtype), SA, tile)
    Bd = dequantize_tiles(decode(QB, dtype), SB, tile)
    return gemm(Ad, Bd, C0, alpha, beta)
