// gemm macro-tile device code for gfx950 (F32 and split-bf16x3):
// C = alpha*A*B + beta*C, row-major.  Shared by the one-problem kernels
// (gemm_tile.hip) and the grouped persistent kernel (batched.hip).
//
// One workgroup computes one BM x BN macro-tile (level-1 tiling, Tiramisu
// paper Sections I and VI-A); inside it each wave owns a (BM/WGM) x (BN/WGN)
// register tile of 32x32 MFMA accumulator blocks (register blocking, level-2
// tiling).  K is walked in BK panels.  Each panel is packed into LDS (array
// packing, Section I) in the operand layout the MFMA reads, with the
// precision conversion done while packing; the next panel's global loads are
// in flight while the MFMAs consume the current one (prefetching), and one
// barrier per panel swaps the two LDS stages (Layer IV synchronisation,
// Section IV).  Tiles that lie wholly inside M x N run an unpredicated body;
// the others run a predicated body (full/partial tile separation,
// Section V-A); the choice is uniform per workgroup, so no wave diverges.
//
// Packing layout.  LDS holds 16-byte "units": KU consecutive k values of one
// row of A (or one column of B).  F32: KU = 4 floats; X3: KU = 8 bf16, kept in
// two arrays (hi and lo parts).  A panel = [BK/KU][BM] units, B panel =
// [BK/KU][BN] units.  For every 2*KU slice of K, lane l of a wave reads unit
// 2g + (l / 32) of row (l % 32) of each of its 32-row blocks: the MFMA's two
// k-halves (lanes 0-31, 32-63) take the two units, and within a unit the k
// order is the element order.  A and B use the same map, so every product
// pairs equal k.  Row indices are XOR-swizzled so that both the packing
// writes and the operand reads hit distinct LDS banks.
#pragma once
#include <hip/hip_runtime.h>

#include "epilogue.h"
#include "kargs.h"

namespace tg {

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
// Four floats at a 4-byte aligned address: one 16-byte load instruction (the
// hardware takes dword-aligned multi-dword loads).
typedef float f32x4u __attribute__((ext_vector_type(4), aligned(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int MODE_, int BM_, int BN_, int BK_, int WGM_, int WGN_, int VEC_>
struct Cfg {
    static constexpr int MODE = MODE_, BM = BM_, BN = BN_, BK = BK_;
    static constexpr int WGM = WGM_, WGN = WGN_, VEC = VEC_;
    static constexpr int NT = 64 * WGM * WGN;
    static constexpr int KU = (MODE == MODE_F32) ? 4 : 8;  // k values per 16-byte unit
    static constexpr int UK = BK / KU;                       // units along K per panel
    static constexpr int WTM = BM / WGM, WTN = BN / WGN;     // wave tile
    static constexpr int TM = WTM / 32, TN = WTN / 32;       // 32x32 blocks per wave
    static constexpr int A_PER_T = BM * UK / NT;             // A units loaded per thread
    // B is loaded as KU k-rows x BVJ columns per thread (transposed while packing).
    static constexpr int BVJ = ((UK * (BN / 4)) % NT == 0) ? 4 : (((UK * (BN / 2)) % NT == 0) ? 2 : 1);
    static constexpr int B_PER_T = UK * (BN / BVJ) / NT;
    static constexpr int NARR = (MODE == MODE_F32) ? 1 : 2;  // hi (+ lo) arrays
    static constexpr int LDS_A = UK * BM * 16;
    static constexpr int LDS_B = UK * BN * 16;
    static constexpr int LDS_STAGE = NARR * (LDS_A + LDS_B);
    static constexpr int LDS_BYTES = 2 * LDS_STAGE;

    static_assert(BK % (2 * KU) == 0, "a panel holds whole 2*KU slices");
    static_assert(WTM % 32 == 0 && WTN % 32 == 0, "wave tiles are whole 32x32 blocks");
    static_assert((BM * UK) % NT == 0 && A_PER_T >= 1, "A units divide among threads");
    static_assert((UK * (BN / BVJ)) % NT == 0 && B_PER_T >= 1, "B tiles divide among threads");
    static_assert(UK <= 16 && (16 % UK) == 0, "A swizzle assumes at most 16 units per row");
    static_assert(BM % 16 == 0 && BN % 64 == 0, "swizzles permute within 16-row groups");
    static_assert((BN / BVJ) >= 16, "16 consecutive lanes pack one B unit row");
    static_assert(LDS_BYTES <= 160 * 1024, "gfx950 LDS is 160 KB per workgroup");
};

// A unit (row r, k-unit u) lives at slot u*BM + swz_a(r, u).  Packing writes
// come from 16 lanes covering 16/UK rows x UK units; XOR with u*(16/UK) makes
// their 16 slots distinct modulo 16, and an operand read (fixed u, 32
// consecutive rows) only permutes rows inside aligned groups of 16.
template <int UK>
__device__ __forceinline__ int swz_a(int r, int u) { return r ^ ((u * (16 / UK)) & 15); }

// B unit (column j) of a k-unit row: 16 packing lanes write columns
// j = BVJ*q + c for 16 consecutive q; XOR of the low bits with bits 4.. of j
// spreads them over 16 slots.  Reads of 32 consecutive columns stay
// conflict-free because the XOR value is constant within 16-column groups.
template <int BVJ>
__device__ __forceinline__ int swz_b(int j) { return j ^ ((j >> 4) & (BVJ - 1)); }

__device__ __forceinline__ void split_bf16(const float x, __bf16& hi, __bf16& lo)
{
    hi = (__bf16)x;                       // round to nearest even
    lo = (__bf16)(x - (float)hi);         // x - hi is exact in float32
}

// The same split of two values at once: one packed conversion (round to
// nearest even, as above) per pair for the high parts and one for the low
// parts; the high parts go back to float32 by moving their bits into place.
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void split_bf16_pair(float x0, float x1, uint32_t& hi, uint32_t& lo)
{
    const bf16x2_t h = __builtin_convertvector(f32x2_t{x0, x1}, bf16x2_t);
    hi = __builtin_bit_cast(uint32_t, h);
    const float h0 = __uint_as_float(hi << 16), h1 = __uint_as_float(hi & 0xffff0000u);
    lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_t{x0 - h0, x1 - h1}, bf16x2_t));
}

// Eight consecutive values x[0..7] into eight high and eight low parts.
template <class X>
__device__ __forceinline__ void split_bf16x8(const X& x, bf16x8& hi, bf16x8& lo)
{
    typedef uint32_t u32v4 __attribute__((ext_vector_type(4)));
    u32v4 h, l;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        uint32_t hh, ll;
        split_bf16_pair(x[2 * e], x[2 * e + 1], hh, ll);
        h[e] = hh;
        l[e] = ll;
    }
    hi = __builtin_bit_cast(bf16x8, h);
    lo = __builtin_bit_cast(bf16x8, l);
}

template <int KU> struct UnitVec;
template <> struct UnitVec<4> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct UnitVec<8> { typedef float type __attribute__((ext_vector_type(8))); };

// Operand geometry of a plain gemm: A and B are the matrices of GemmArgs.
struct NoGeom {};

template <class CF>
struct Panel {
    static constexpr int KU = CF::KU, UK = CF::UK, NT = CF::NT, BM = CF::BM, BN = CF::BN;
    static constexpr int BVJ = CF::BVJ;
    typedef typename UnitVec<KU>::type fu;  // the KU float32 values of one unit
    using Geom = NoGeom;

    fu ra[CF::A_PER_T];          // A: one unit (row r, k-unit u) per entry
    fu rb[CF::B_PER_T][BVJ];     // B: already transposed, one unit per column

    // Per-tile set-up of the loads (none for a plain gemm).
    __device__ __forceinline__ void init(const GemmArgs&, int, int, const Geom&) {}

    // Global -> registers for the panel starting at k0.  PRED: per-element
    // bounds checks (partial tiles and the K remainder); out-of-range
    // elements load as zero and are never dereferenced.
    template <bool PRED>
    __device__ __forceinline__ void load(const GemmArgs& a, int m0, int n0, int k0, int t, const Geom&)
    {
        load_a<PRED>(a, m0, k0, t);
        load_b<PRED>(a, n0, k0, t);
    }

    template <bool PRED>
    __device__ __forceinline__ void load_a(const GemmArgs& a, int m0, int k0, int t)
    {
        const float* A = static_cast<const float*>(a.A);
#pragma unroll
        for (int p = 0; p < CF::A_PER_T; ++p) {
            const int q = t + p * NT;
            const int r = q / UK, u = q % UK;
            const int kb = k0 + u * KU;
            const float* src = A + (int64_t)(m0 + r) * a.lda + kb;
            if (!PRED) {
                if (CF::VEC == 4) {
#pragma unroll
                    for (int c = 0; c < KU / 4; ++c) {
                        const f32x4 v = *reinterpret_cast<const f32x4*>(src + 4 * c);
#pragma unroll
                        for (int e = 0; e < 4; ++e) ra[p][4 * c + e] = v[e];
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < KU; ++e) ra[p][e] = src[e];
                }
            } else {
                const bool row_ok = (m0 + r) < a.M;
#pragma unroll
                for (int e = 0; e < KU; ++e) {
                    float v = 0.f;
                    if (row_ok && kb + e < a.K) v = src[e];
                    ra[p][e] = v;
                }
            }
        }
    }

    template <bool PRED>
    __device__ __forceinline__ void load_b(const GemmArgs& a, int n0, int k0, int t)
    {
        const float* B = static_cast<const float*>(a.B);
#pragma unroll
        for (int p = 0; p < CF::B_PER_T; ++p) {
            const int q = t + p * NT;
            const int jq = q % (BN / BVJ), u = q / (BN / BVJ);
            const int n = n0 + jq * BVJ;
#pragma unroll
            for (int e = 0; e < KU; ++e) {
                const int k = k0 + u * KU + e;
                const float* src = B + (int64_t)k * a.ldb + n;
                if (!PRED) {
                    if (CF::VEC == 4 && BVJ == 4) {
                        const f32x4 v = *reinterpret_cast<const f32x4*>(src);
#pragma unroll
                        for (int c = 0; c < BVJ; ++c) rb[p][c][e] = v[c];
                    } else if (CF::VEC == 4 && BVJ == 2) {
                        const f32x2 v = *reinterpret_cast<const f32x2*>(src);
#pragma unroll
                        for (int c = 0; c < BVJ; ++c) rb[p][c][e] = v[c];
                    } else {
#pragma unroll
                        for (int c = 0; c < BVJ; ++c) rb[p][c][e] = src[c];
                    }
                } else {
                    const bool k_ok = k < a.K;
#pragma unroll
                    for (int c = 0; c < BVJ; ++c) {
                        float v = 0.f;
                        if (k_ok && n + c < a.N) v = src[c];
                        rb[p][c][e] = v;
                    }
                }
            }
        }
    }

    // Registers -> LDS stage (packing; the precision split happens here).
    __device__ __forceinline__ void store(char* stage, int t) const
    {
        char* a_hi = stage;
        char* a_lo = stage + CF::LDS_A;  // X3 only
        char* b_hi = stage + CF::NARR * CF::LDS_A;
        char* b_lo = b_hi + CF::LDS_B;   // X3 only
#pragma unroll
        for (int p = 0; p < CF::A_PER_T; ++p) {
            const int q = t + p * NT;
            const int r = q / UK, u = q % UK;
            const int slot = u * BM + swz_a<UK>(r, u);
            put_unit(a_hi, a_lo, slot, ra[p]);
        }
#pragma unroll
        for (int p = 0; p < CF::B_PER_T; ++p) {
            const int q = t + p * NT;
            const int jq = q % (BN / BVJ), u = q / (BN / BVJ);
#pragma unroll
            for (int c = 0; c < BVJ; ++c) {
                const int j = jq * BVJ + c;
                put_unit(b_hi, b_lo, u * BN + swz_b<BVJ>(j), rb[p][c]);
            }
        }
    }

    __device__ __forceinline__ static void put_unit(char* hi_arr, char* lo_arr, int slot, const fu& x)
    {
        if (CF::MODE == MODE_F32) {
            *reinterpret_cast<fu*>(hi_arr + slot * 16) = x;
        } else {
            bf16x8 h, l;
            split_bf16x8(x, h, l);
            *reinterpret_cast<bf16x8*>(hi_arr + slot * 16) = h;
            *reinterpret_cast<bf16x8*>(lo_arr + slot * 16) = l;
        }
    }
};

// MFMA over one LDS stage into the wave's accumulator blocks.
template <class CF>
__device__ __forceinline__ void mma_stage(const char* stage, f32x16 (&acc)[CF::TM][CF::TN],
                                          int wm0, int wn0, int lane)
{
    constexpr int UK = CF::UK, BM = CF::BM, BN = CF::BN, TM = CF::TM, TN = CF::TN;
    const char* a_hi = stage;
    const char* a_lo = stage + CF::LDS_A;
    const char* b_hi = stage + CF::NARR * CF::LDS_A;
    const char* b_lo = b_hi + CF::LDS_B;
    const int h = lane >> 5, l32 = lane & 31;
#pragma unroll
    for (int g = 0; g < UK / 2; ++g) {
        const int u = 2 * g + h;
        if (CF::MODE == MODE_F32) {
            f32x4 av[TM], bv[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i)
                av[i] = *reinterpret_cast<const f32x4*>(
                    a_hi + (u * BM + swz_a<UK>(wm0 + 32 * i + l32, u)) * 16);
#pragma unroll
            for (int j = 0; j < TN; ++j)
                bv[j] = *reinterpret_cast<const f32x4*>(
                    b_hi + (u * BN + swz_b<CF::BVJ>(wn0 + 32 * j + l32)) * 16);
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i][s], bv[j][s],
                                                                         acc[i][j], 0, 0, 0);
        } else {
            bf16x8 ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const int off = (u * BM + swz_a<UK>(wm0 + 32 * i + l32, u)) * 16;
                ah[i] = *reinterpret_cast<const bf16x8*>(a_hi + off);
                al[i] = *reinterpret_cast<const bf16x8*>(a_lo + off);
            }
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int off = (u * BN + swz_b<CF::BVJ>(wn0 + 32 * j + l32)) * 16;
                bh[j] = *reinterpret_cast<const bf16x8*>(b_hi + off);
                bl[j] = *reinterpret_cast<const bf16x8*>(b_lo + off);
            }
            // small terms first: lo*hi, hi*lo, then hi*hi
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
        }
    }
}

// PN: the operand loader (Panel for a plain gemm; a loader with its own Geom
// can compute A's addresses differently, e.g. the implicit im2col of a
// convolution, and share the rest of the body).
template <class CF, bool EDGE, class PN = Panel<CF>>
__device__ __forceinline__ void tile_body(const GemmArgs& a, int m0, int n0, char* lds,
                                          const typename PN::Geom& geom = typename PN::Geom())
{
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int wm0 = (wave / CF::WGN) * CF::WTM;
    const int wn0 = (wave % CF::WGN) * CF::WTN;

    f32x16 acc[CF::TM][CF::TN];
#pragma unroll
    for (int i = 0; i < CF::TM; ++i)
#pragma unroll
        for (int j = 0; j < CF::TN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    const int nfull = a.K / CF::BK;                      // panels with no K remainder
    const int npanel = (a.K + CF::BK - 1) / CF::BK;

    PN pn;
    pn.init(a, m0, t, geom);
    if (!EDGE && nfull > 0) pn.template load<false>(a, m0, n0, 0, t, geom);
    else pn.template load<true>(a, m0, n0, 0, t, geom);
    pn.store(lds, t);
    __syncthreads();

    for (int s = 0; s < npanel; ++s) {
        const int nx = s + 1;
        if (nx < npanel) {
            if (!EDGE && nx < nfull) pn.template load<false>(a, m0, n0, nx * CF::BK, t, geom);
            else pn.template load<true>(a, m0, n0, nx * CF::BK, t, geom);
        }
        mma_stage<CF>(lds + (s & 1) * CF::LDS_STAGE, acc, wm0, wn0, lane);
        if (nx < npanel) pn.store(lds + (nx & 1) * CF::LDS_STAGE, t);
        __syncthreads();
    }

    // Fused epilogue: C = alpha*acc + beta*C; beta == 0 never reads C.
    // 32x32 accumulator layout: register r of lane l holds
    // row 8*(r/4) + 4*(l/32) + r%4, column l%32 of the block.
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

}  // namespace tg
