// Low-precision gemm with one float32 scale per 128 x 128 tile (project
// addition; the Tiramisu paper computes gemm in single precision), and the
// per-tile quantiser that produces such inputs.
//
//   C = alpha * sum_kb sA[i/128, kb] * sB[kb, j/128] * (sum_{k in kb} qA[i,k] qB[k,j])
//       + beta * C
//
// The structure is the one of the float32 kernels (gemm_tile.hip): macro-tile
// per workgroup, wave register tiles of 32x32 MFMA blocks, K panels packed into
// double-buffered LDS in the MFMA operand layout, predicated partial tiles.
// Differences:
//   - the inputs are already bf16 or OCP E4M3FN codes, so packing moves bytes
//     (B is transposed in registers with byte permutes so that every LDS unit
//     holds consecutive k of one column);
//   - a panel never straddles a 128-wide K scale block (128 % BK == 0), and
//     each 32x32 block lies inside one 128 x 128 scale tile of C, so a block's
//     products for one K scale block sum into a partial accumulator that is
//     folded into the running sum with the single factor sA * sB.
// MFMA: v_mfma_f32_32x32x16_bf16 and v_mfma_f32_32x32x64_f8f6f4 (e4m3 x e4m3).
#include <hip/hip_runtime.h>

#include "epilogue.h"
#include "kargs.h"
#include "registry.h"
#include "../../include/tgemm.h"

namespace tg {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kScaleTile = 128;

template <int MODE_, int BM_, int BN_, int BK_, int WGM_, int WGN_, int VEC_>
struct SCfg {
    static constexpr int MODE = MODE_, BM = BM_, BN = BN_, BK = BK_;
    static constexpr int WGM = WGM_, WGN = WGN_, VEC = VEC_;
    static constexpr int NT = 64 * WGM * WGN;
    static constexpr int ES = (MODE == MODE_BF16) ? 2 : 1;   // bytes per element
    static constexpr int KU = 16 / ES;                       // k values per 16-byte unit
    static constexpr int UK = BK / KU;                       // units along K per panel
    static constexpr int MK = (MODE == MODE_BF16) ? 16 : 64; // k per MFMA
    static constexpr int UPL = MK / KU / 2;                  // units per lane per MFMA
    static constexpr int NG = BK / MK;                       // MFMAs per block per panel
    static constexpr int WTM = BM / WGM, WTN = BN / WGN;
    static constexpr int TM = WTM / 32, TN = WTN / 32;
    static constexpr int A_PER_T = BM * UK / NT;
    static constexpr int BVJ = 4 / ES;                       // B columns per 4-byte load
    static constexpr int B_PER_T = UK * (BN / BVJ) / NT;
    static constexpr int LDS_A = UK * BM * 16;
    static constexpr int LDS_B = UK * BN * 16;
    static constexpr int LDS_STAGE = LDS_A + LDS_B;
    static constexpr int LDS_BYTES = 2 * LDS_STAGE;

    static_assert(kScaleTile % BK == 0 && BK % MK == 0, "panels tile the 128-wide K scale blocks");
    static_assert(kScaleTile % 32 == 0, "32x32 blocks lie inside one scale tile");
    static_assert(WTM % 32 == 0 && WTN % 32 == 0, "wave tiles are whole 32x32 blocks");
    static_assert((BM * UK) % NT == 0 && A_PER_T >= 1, "A units divide among threads");
    static_assert((UK * (BN / BVJ)) % NT == 0 && B_PER_T >= 1, "B tiles divide among threads");
    static_assert(UK <= 16 && (16 % UK) == 0, "A swizzle assumes at most 16 units per row");
    static_assert(BM % 16 == 0 && BN % 64 == 0 && (BN / BVJ) >= 16, "swizzle groups");
    static_assert(LDS_BYTES <= 160 * 1024, "gfx950 LDS is 160 KB per workgroup");
};

template <int UK>
__device__ __forceinline__ int sswz_a(int r, int u) { return r ^ ((u * (16 / UK)) & 15); }
template <int BVJ>
__device__ __forceinline__ int sswz_b(int j) { return j ^ ((j >> 4) & (BVJ - 1)); }

template <int ES>
__device__ __forceinline__ uint32_t load_elem(const uint8_t* p)
{
    if (ES == 2) return *reinterpret_cast<const uint16_t*>(p);
    return *p;
}

template <class CF>
struct SPanel {
    static constexpr int ES = CF::ES, KU = CF::KU, UK = CF::UK, NT = CF::NT;
    static constexpr int BM = CF::BM, BN = CF::BN, BVJ = CF::BVJ;

    u32x4 ra[CF::A_PER_T];
    uint32_t rb[CF::B_PER_T][KU];  // KU rows x one dword (BVJ columns) each

    template <bool PRED>
    __device__ __forceinline__ void load(const GemmArgs& a, int m0, int n0, int k0, int t)
    {
        const uint8_t* A = static_cast<const uint8_t*>(a.A);
        const uint8_t* B = static_cast<const uint8_t*>(a.B);
#pragma unroll
        for (int p = 0; p < CF::A_PER_T; ++p) {
            const int q = t + p * NT;
            const int r = q / UK, u = q % UK;
            const int kb = k0 + u * KU;
            const uint8_t* src = A + ((int64_t)(m0 + r) * a.lda + kb) * ES;
            if (!PRED && CF::VEC == 4) {
                ra[p] = *reinterpret_cast<const u32x4*>(src);
            } else {
                const bool row_ok = !PRED || (m0 + r) < a.M;
                uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
                for (int e = 0; e < KU; ++e) {
                    uint32_t v = 0u;
                    if (row_ok && (!PRED || kb + e < a.K)) v = load_elem<ES>(src + e * ES);
                    w[(e * ES) / 4] |= v << (8 * ((e * ES) % 4));
                }
                ra[p] = u32x4{w[0], w[1], w[2], w[3]};
            }
        }
#pragma unroll
        for (int p = 0; p < CF::B_PER_T; ++p) {
            const int q = t + p * NT;
            const int jq = q % (BN / BVJ), u = q / (BN / BVJ);
            const int n = n0 + jq * BVJ;
#pragma unroll
            for (int e = 0; e < KU; ++e) {
                const int k = k0 + u * KU + e;
                const uint8_t* src = B + ((int64_t)k * a.ldb + n) * ES;
                if (!PRED && CF::VEC == 4) {
                    rb[p][e] = *reinterpret_cast<const uint32_t*>(src);
                } else {
                    uint32_t w = 0u;
#pragma unroll
                    for (int c = 0; c < BVJ; ++c) {
                        if (!PRED || (k < a.K && n + c < a.N))
                            w |= load_elem<ES>(src + c * ES) << (8 * ES * c);
                    }
                    rb[p][e] = w;
                }
            }
        }
    }

    // Column c of a KU x BVJ register tile as one unit (KU consecutive k).
    __device__ __forceinline__ u32x4 column_unit(int p, int c) const
    {
        u32x4 out;
        if (ES == 2) {
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                const uint32_t lo = (rb[p][2 * d] >> (16 * c)) & 0xffffu;
                const uint32_t hi = (rb[p][2 * d + 1] >> (16 * c)) & 0xffffu;
                out[d] = lo | (hi << 16);
            }
        } else {
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                uint32_t w = 0u;
#pragma unroll
                for (int b = 0; b < 4; ++b) w |= ((rb[p][4 * d + b] >> (8 * c)) & 0xffu) << (8 * b);
                out[d] = w;
            }
        }
        return out;
    }

    __device__ __forceinline__ void store(char* stage, int t) const
    {
        char* la = stage;
        char* lb = stage + CF::LDS_A;
#pragma unroll
        for (int p = 0; p < CF::A_PER_T; ++p) {
            const int q = t + p * NT;
            const int r = q / UK, u = q % UK;
            *reinterpret_cast<u32x4*>(la + (u * BM + sswz_a<UK>(r, u)) * 16) = ra[p];
        }
#pragma unroll
        for (int p = 0; p < CF::B_PER_T; ++p) {
            const int q = t + p * NT;
            const int jq = q % (BN / BVJ), u = q / (BN / BVJ);
#pragma unroll
            for (int c = 0; c < BVJ; ++c) {
                const int j = jq * BVJ + c;
                *reinterpret_cast<u32x4*>(lb + (u * BN + sswz_b<BVJ>(j)) * 16) = column_unit(p, c);
            }
        }
    }
};

template <class CF>
__device__ __forceinline__ void mma_panel(const char* stage, f32x16 (&part)[CF::TM][CF::TN],
                                          int wm0, int wn0, int lane)
{
    constexpr int UK = CF::UK, BM = CF::BM, BN = CF::BN, UPL = CF::UPL;
    const char* la = stage;
    const char* lb = stage + CF::LDS_A;
    const int h = lane >> 5, l32 = lane & 31;
#pragma unroll
    for (int g = 0; g < CF::NG; ++g) {
        u32x4 av[CF::TM][UPL], bv[CF::TN][UPL];
#pragma unroll
        for (int v = 0; v < UPL; ++v) {
            const int u = (2 * g + h) * UPL + v;
#pragma unroll
            for (int i = 0; i < CF::TM; ++i)
                av[i][v] = *reinterpret_cast<const u32x4*>(
                    la + (u * BM + sswz_a<UK>(wm0 + 32 * i + l32, u)) * 16);
#pragma unroll
            for (int j = 0; j < CF::TN; ++j)
                bv[j][v] = *reinterpret_cast<const u32x4*>(
                    lb + (u * BN + sswz_b<CF::BVJ>(wn0 + 32 * j + l32)) * 16);
        }
#pragma unroll
        for (int i = 0; i < CF::TM; ++i)
#pragma unroll
            for (int j = 0; j < CF::TN; ++j) {
                if (CF::MODE == MODE_BF16) {
                    const bf16x8 x = __builtin_bit_cast(bf16x8, av[i][0]);
                    const bf16x8 y = __builtin_bit_cast(bf16x8, bv[j][0]);
                    part[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, y, part[i][j], 0, 0, 0);
                } else {
                    const i32x8 x = {(int)av[i][0][0], (int)av[i][0][1], (int)av[i][0][2],
                                     (int)av[i][0][3], (int)av[i][UPL - 1][0], (int)av[i][UPL - 1][1],
                                     (int)av[i][UPL - 1][2], (int)av[i][UPL - 1][3]};
                    const i32x8 y = {(int)bv[j][0][0], (int)bv[j][0][1], (int)bv[j][0][2],
                                     (int)bv[j][0][3], (int)bv[j][UPL - 1][0], (int)bv[j][UPL - 1][1],
                                     (int)bv[j][UPL - 1][2], (int)bv[j][UPL - 1][3]};
                    // format codes 0/0: both operands OCP e4m3; no block scaling
                    part[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                        x, y, part[i][j], 0, 0, 0, 0, 0, 0);
                }
            }
    }
}

template <class CF, bool EDGE>
__device__ __forceinline__ void scaled_body(const GemmArgs& a, int m0, int n0, char* lds)
{
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int wm0 = (wave / CF::WGN) * CF::WTM;
    const int wn0 = (wave % CF::WGN) * CF::WTN;

    f32x16 acc[CF::TM][CF::TN], part[CF::TM][CF::TN];
#pragma unroll
    for (int i = 0; i < CF::TM; ++i)
#pragma unroll
        for (int j = 0; j < CF::TN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                acc[i][j][r] = 0.f;
                part[i][j][r] = 0.f;
            }

    const int nfull = a.K / CF::BK;
    const int npanel = (a.K + CF::BK - 1) / CF::BK;

    SPanel<CF> pn;
    if (!EDGE && nfull > 0) pn.template load<false>(a, m0, n0, 0, t);
    else pn.template load<true>(a, m0, n0, 0, t);
    pn.store(lds, t);
    __syncthreads();

    for (int s = 0; s < npanel; ++s) {
        const int nx = s + 1;
        if (nx < npanel) {
            if (!EDGE && nx < nfull) pn.template load<false>(a, m0, n0, nx * CF::BK, t);
            else pn.template load<true>(a, m0, n0, nx * CF::BK, t);
        }
        mma_panel<CF>(lds + (s & 1) * CF::LDS_STAGE, part, wm0, wn0, lane);
        const int kend = (s + 1) * CF::BK;
        if (kend % kScaleTile == 0 || nx == npanel) {
            // fold the partial sums of this K scale block
            const int kb = (s * CF::BK) / kScaleTile;
#pragma unroll
            for (int i = 0; i < CF::TM; ++i) {
                const int row0 = m0 + wm0 + 32 * i;
#pragma unroll
                for (int j = 0; j < CF::TN; ++j) {
                    const int col0 = n0 + wn0 + 32 * j;
                    float sc = 1.f;
                    if (a.sA) {
                        sc = 0.f;
                        if (!EDGE || (row0 < a.M && col0 < a.N))
                            sc = a.sA[(int64_t)(row0 / kScaleTile) * a.lds_a + kb] *
                                 a.sB[(int64_t)kb * a.lds_b + col0 / kScaleTile];
                    }
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        acc[i][j][r] = fmaf(sc, part[i][j][r], acc[i][j][r]);
                        part[i][j][r] = 0.f;
                    }
                }
            }
        }
        if (nx < npanel) pn.store(lds + (nx & 1) * CF::LDS_STAGE, t);
        __syncthreads();
    }

    const int h = lane >> 5, l32 = lane & 31;
    write_c<CF::TM, CF::TN, 16>(
        a.C, a.ldc, a.M, a.N, a.beta, 4 * h, l32,
        [&](int i, int j, float (&v)[16]) {
#pragma unroll
            for (int r = 0; r < 16; ++r) v[r] = a.alpha * acc[i][j][r];
        },
        [&](int i, int j, int& r0, int& c0) {
            r0 = m0 + wm0 + 32 * i;
            c0 = n0 + wn0 + 32 * j;
        },
        [](int r) { return 8 * (r >> 2) + (r & 3); });
}

template <class CF>
__global__ void __launch_bounds__(CF::NT) scaled_kernel(GemmArgs a)
{
    __shared__ __attribute__((aligned(16))) char lds[CF::LDS_BYTES];
    const TileCoord tc = map_tile(blockIdx.x, a.tiles_m, a.tiles_n, a.group_m, a.xcd_remap);
    const int m0 = tc.tm * CF::BM, n0 = tc.tn * CF::BN;
    const bool full = (m0 + CF::BM <= a.M) && (n0 + CF::BN <= a.N);
    if (full) scaled_body<CF, false>(a, m0, n0, lds);
    else scaled_body<CF, true>(a, m0, n0, lds);
}

// ------------------------------------------------------------------ quantiser
// Nearest E4M3FN code of y (ties to even), saturating at +-448.  Normal range:
// y = m * 2^e, the grid step is 2^(e-3); subnormal range (|y| < 2^-6): step
// 2^-9.  Scaling by a power of two is exact in float32 and rint rounds half to
// even, so rint(|y| / step) is the correctly rounded mantissa count; a carry
// to 16 moves into the next exponent through the code arithmetic.
__device__ __forceinline__ uint32_t e4m3_code(float y)
{
    const uint32_t sign = (__float_as_uint(y) >> 24) & 0x80u;
    const float a = fminf(fabsf(y), 448.f);
    uint32_t code;
    if (a < 0.015625f) {
        code = (uint32_t)__builtin_rintf(a * 512.f);
    } else {
        const int e = (int)((__float_as_uint(a) >> 23) & 0xffu) - 127;  // floor(log2 a)
        const float step_inv = __uint_as_float((uint32_t)(127 + 3 - e) << 23);
        const uint32_t q = (uint32_t)__builtin_rintf(a * step_inv);    // 8 .. 16
        code = ((uint32_t)(e + 7) << 3) + (q - 8u);
    }
    return code | sign;
}

// One workgroup per 128 x 128 tile, one read of X: the tile is held in
// registers (64 values per thread), its amax found by a block reduction, and
// the codes written from the registers.  Thread t covers columns 4*(t % 32)
// .. +3 of rows t / 32 + 8p, p = 0..15, so a wave reads two whole 512-byte
// tile rows per load and writes them back as two runs of codes.  vec: X rows
// allow 16-byte loads and Q rows 4-byte (e4m3) or 8-byte (bf16) stores.
__global__ void __launch_bounds__(256) quantize_kernel(int rows, int cols, const float* X,
                                                       int64_t ldx, void* Q, int64_t ldq,
                                                       float* S, int grid_cols, int dtype, int vec)
{
    __shared__ float red[4];
    const int tile = blockIdx.x;
    const int r0 = (tile / grid_cols) * kScaleTile, c0 = (tile % grid_cols) * kScaleTile;
    const int t = threadIdx.x;
    const int c = c0 + 4 * (t & 31), rt = r0 + (t >> 5);
    const bool full = vec && r0 + kScaleTile <= rows && c0 + kScaleTile <= cols;
    float v[16][4];
    if (full) {
#pragma unroll
        for (int p = 0; p < 16; ++p) {
            const f32x4 x = __builtin_nontemporal_load(
                reinterpret_cast<const f32x4*>(X + (int64_t)(rt + 8 * p) * ldx + c));
#pragma unroll
            for (int e = 0; e < 4; ++e) v[p][e] = x[e];
        }
    } else {
#pragma unroll
        for (int p = 0; p < 16; ++p)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                v[p][e] = (rt + 8 * p < rows && c + e < cols) ? X[(int64_t)(rt + 8 * p) * ldx + c + e] : 0.f;
    }
    float m = 0.f;
#pragma unroll
    for (int p = 0; p < 16; ++p)
#pragma unroll
        for (int e = 0; e < 4; ++e) m = fmaxf(m, fabsf(v[p][e]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    if ((t & 63) == 0) red[t >> 6] = m;
    __syncthreads();
    const float amax = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    // power-of-two scales (exact divisions; the e4m3 matrix core applies them
    // as block scales): e4m3 the power of two with amax / s in (224, 448]
    // (448 = 0.875 * 2^9), bf16 2^ceil(log2 amax)
    float s = 1.f;
    if (amax > 0.f) {
        int e;
        const float f = frexpf(amax, &e);  // amax = f * 2^e, 0.5 <= f < 1
        if (dtype == TGEMM_FP8_E4M3) {
            e = f <= 0.875f ? e - 9 : e - 8;
            s = ldexpf(1.f, e < -126 ? -126 : (e > 127 ? 127 : e));
        } else {
            s = ldexpf(1.f, f == 0.5f ? e - 1 : e);
        }
    }
    if (t == 0) S[tile] = s;
#pragma unroll
    for (int p = 0; p < 16; ++p) {
        const int r = rt + 8 * p;
        if (!full && r >= rows) continue;
        if (dtype == TGEMM_FP8_E4M3) {
            uint32_t q[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) q[e] = e4m3_code(v[p][e] / s);
            uint8_t* dst = static_cast<uint8_t*>(Q) + (int64_t)r * ldq + c;
            if (full) {
                *reinterpret_cast<uint32_t*>(dst) = q[0] | (q[1] << 8) | (q[2] << 16) | (q[3] << 24);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (c + e < cols) dst[e] = (uint8_t)q[e];
            }
        } else {
            __bf16 q[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) q[e] = (__bf16)(v[p][e] / s);
            __bf16* dst = static_cast<__bf16*>(Q) + (int64_t)r * ldq + c;
            if (full) {
                uint32_t w[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) w[e] = __builtin_bit_cast(uint16_t, q[e]);
                *reinterpret_cast<uint2*>(dst) = make_uint2(w[0] | (w[1] << 16), w[2] | (w[3] << 16));
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (c + e < cols) dst[e] = q[e];
            }
        }
    }
}

hipError_t launch_quantize(int rows, int cols, const float* X, int64_t ldx, void* Q, int64_t ldq,
                           float* S, int dtype, hipStream_t s)
{
    const int gr = (rows + kScaleTile - 1) / kScaleTile, gc = (cols + kScaleTile - 1) / kScaleTile;
    const int64_t qes = dtype == TGEMM_FP8_E4M3 ? 1 : 2;
    const int vec = reinterpret_cast<uintptr_t>(X) % 16 == 0 && ldx % 4 == 0 &&
                    reinterpret_cast<uintptr_t>(Q) % (4 * qes) == 0 && ldq % 4 == 0;
    hipLaunchKernelGGL(quantize_kernel, dim3((unsigned)(gr * gc)), dim3(256), 0, s, rows, cols, X,
                       ldx, Q, ldq, S, gc, dtype, vec);
    return hipGetLastError();
}

#define TG_SSCHED(DT, MODE, BM, BN, BK, WGM, WGN, VEC)                                        \
    {DT, BM, BN, BK, WGM, WGN, VEC, SCfg<MODE, BM, BN, BK, WGM, WGN, VEC>::LDS_BYTES,         \
     SCfg<MODE, BM, BN, BK, WGM, WGN, VEC>::NT, &scaled_kernel<SCfg<MODE, BM, BN, BK, WGM, WGN, VEC>>}

#define TG_SSCHED_V(DT, MODE, BM, BN, BK, WGM, WGN) \
    TG_SSCHED(DT, MODE, BM, BN, BK, WGM, WGN, 4), TG_SSCHED(DT, MODE, BM, BN, BK, WGM, WGN, 1)

static const SchedDesc kScaledSchedules[] = {
    TG_SSCHED_V(TGEMM_BF16, MODE_BF16, 128, 128, 64, 2, 2),
    TG_SSCHED_V(TGEMM_BF16, MODE_BF16, 128, 128, 128, 2, 2),
    TG_SSCHED_V(TGEMM_BF16, MODE_BF16, 64, 64, 64, 2, 2),
    TG_SSCHED_V(TGEMM_FP8_E4M3, MODE_FP8, 128, 128, 128, 2, 2),
    TG_SSCHED_V(TGEMM_FP8_E4M3, MODE_FP8, 256, 128, 128, 2, 2),
    TG_SSCHED_V(TGEMM_FP8_E4M3, MODE_FP8, 64, 128, 128, 2, 2),
};

const SchedDesc* scaled_schedules(int* n)
{
    *n = (int)(sizeof(kScaledSchedules) / sizeof(kScaledSchedules[0]));
    return kScaledSchedules;
}

}  // namespace tg
