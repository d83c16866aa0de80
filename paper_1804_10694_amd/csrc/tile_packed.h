// Device code of the packed-operand gemm (all MFMA forms): the K-panel
// pipeline from packed, K-contiguous operand buffers into LDS and the MFMA
// register tiles, for one macro-tile.  Shared by the one-problem packed
// kernels (gemm_packed.hip) and the grouped launch (batched.hip).
//
// Packing (Tiramisu paper, Section I, array packing after Goto and van de
// Geijn): A (M x K) and B (K x N), row-major, are copied into buffers whose
// rows are K-contiguous, in the element type the MFMA reads:
//   Ap[m][k] = conv(A[m][k]),   Bp[n][k] = conv(B[k][n])   (B transposed)
// where conv is the x3 split (two arrays, hi and lo) or a plain copy of the
// values (f32) or codes (bf16, e4m3).  Rows are padded to whole macro-tiles
// and K to whole panels, with zeros, so the main loop's loads carry no
// predicates; full/partial tiles (Section V-A) differ only in the epilogue.
//
// Main loop: K panels of BK go from the packed buffers straight into LDS with
// buffer_load ... lds (16 bytes per lane, no register staging); NS stages,
// NS - 1 panels in flight, one barrier per panel.  LDS rows hold a panel's
// 16-byte units of one packed row, XOR-swizzled so that the MFMA operand
// reads of 16 consecutive rows hit distinct banks.
//
// Scaled forms: the running sum is kept divided by the current K block's
// scale product and rescaled when the K block changes:
// acc <- acc * (s_prev / s_cur) at each 128-wide K block, C = alpha * s_last * acc.
#pragma once
#include <hip/hip_runtime.h>

#include "kargs.h"
#include "tile_f32x3.h"

namespace tg {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

// ------------------------------------------------------------------ packing
// Element bytes of the source matrices: float for f32 and x3, codes for bf16
// and e4m3.
template <int MODE>
constexpr int src_bytes() { return MODE == MODE_FP8 ? 1 : MODE == MODE_BF16 ? 2 : 4; }

// Host side: whether rows of X (element size es bytes, row stride ld
// elements) allow the vector loads of pack_row_group (8 elements, 16-byte
// loads; 8 bytes for 1-byte codes) and of pack_col_block (4 elements).
inline int pack_rows_vec(const void* X, int64_t ld, int es)
{
    const int64_t need = es == 1 ? 8 : 16;
    return (reinterpret_cast<uintptr_t>(X) % need == 0) && ((ld * es) % need == 0);
}
inline int pack_cols_vec(const void* X, int64_t ld, int es)
{
    const int64_t need = 4 * es;
    return (reinterpret_cast<uintptr_t>(X) % need == 0) && ((ld * es) % need == 0);
}

// A-side, one group of 8 consecutive k of row r: X (R x K, row stride ldx)
// -> P (row stride Kp); zero beyond R and K.  x3: X is float, P / Plo receive
// the bf16 hi and lo parts.  f32: floats, copied.  bf16 / e4m3: X holds codes,
// copied.  A group wholly inside the matrix takes vector loads: float rows
// always (two 16-byte loads at any 4-byte alignment), code rows when vec says
// X and its row stride allow one 8-element vector load (16-byte aligned rows;
// 8-byte for e4m3).
template <int MODE>
__device__ __forceinline__ void pack_row_group(const void* X, int64_t ldx, int R, int K, void* P,
                                               void* Plo, int Kp, int r, int k0, bool vec)
{
    constexpr int ES = src_bytes<MODE>();
    const bool whole = (ES == 4 || vec) && r < R && k0 + 8 <= K;
    const char* src = static_cast<const char*>(X) + ((int64_t)r * ldx + k0) * ES;
    const int64_t o = (int64_t)r * Kp + k0;
    if (MODE == MODE_F32 || MODE == MODE_X3) {
        f32x4 v0, v1;
        if (whole) {
            v0 = *reinterpret_cast<const f32x4u*>(src);
            v1 = *reinterpret_cast<const f32x4u*>(src + 16);
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const float v = (r < R && k0 + e < K) ? reinterpret_cast<const float*>(src)[e] : 0.f;
                if (e < 4) v0[e] = v;
                else v1[e - 4] = v;
            }
        }
        if (MODE == MODE_F32) {
            float* dst = static_cast<float*>(P) + o;
            *reinterpret_cast<f32x4*>(dst) = v0;
            *reinterpret_cast<f32x4*>(dst + 4) = v1;
        } else {
            bf16x8 h, l;
            const float x[8] = {v0[0], v0[1], v0[2], v0[3], v1[0], v1[1], v1[2], v1[3]};
            split_bf16x8(x, h, l);
            *reinterpret_cast<bf16x8*>(static_cast<__bf16*>(P) + o) = h;
            *reinterpret_cast<bf16x8*>(static_cast<__bf16*>(Plo) + o) = l;
        }
    } else if (MODE == MODE_BF16) {
        u32x4 w;
        if (whole) {
            w = *reinterpret_cast<const u32x4*>(src);
        } else {
            uint32_t c[8];
#pragma unroll
            for (int e = 0; e < 8; ++e)
                c[e] = (r < R && k0 + e < K) ? reinterpret_cast<const uint16_t*>(src)[e] : 0u;
            w = u32x4{c[0] | (c[1] << 16), c[2] | (c[3] << 16), c[4] | (c[5] << 16), c[6] | (c[7] << 16)};
        }
        *reinterpret_cast<u32x4*>(static_cast<uint16_t*>(P) + o) = w;
    } else {
        uint2 w;
        if (whole) {
            w = *reinterpret_cast<const uint2*>(src);
        } else {
            uint32_t w0 = 0, w1 = 0;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const uint32_t v = (r < R && k0 + e < K) ? reinterpret_cast<const uint8_t*>(src)[e] : 0u;
                if (e < 4) w0 |= v << (8 * e);
                else w1 |= v << (8 * (e - 4));
            }
            w = make_uint2(w0, w1);
        }
        *reinterpret_cast<uint2*>(static_cast<uint8_t*>(P) + o) = w;
    }
}

// B-side, one 64 x 64 block (n0, k0): X (K x N, row stride ldx) -> P (row
// stride Kp) = X^T, through the LDS `tile` (x3 and f32: float values; codes
// widened to 32 bits).  Reads: 16 lanes cover 64 consecutive n of one k row,
// four elements each (one vector load when vec and the four lie inside the
// matrix); writes: each lane stores 16 consecutive k of one packed row with
// 16-byte stores.  Zero beyond K and N; nothing written at or beyond Np, and
// Kp must be a multiple of 16.  256 threads; ends with a barrier, so `tile`
// can be reused at once.  Four elements inside the matrix take one vector
// load: floats always (16 bytes at any 4-byte alignment), codes when vec says
// the rows of X are aligned for it.
template <int MODE>
__device__ __forceinline__ void pack_col_block(const void* X, int64_t ldx, int K, int N, void* P,
                                               void* Plo, int Np, int Kp, int n0, int k0,
                                               float (&tile)[64][65], bool vec)
{
    constexpr int ES = src_bytes<MODE>();
    const int t = threadIdx.x;
    {
        const int n4 = t & 15, kr = t >> 4;  // 16 x 16 threads; 4 passes over 64 rows
        const int n = n0 + 4 * n4;
#pragma unroll
        for (int pass = 0; pass < 4; ++pass) {
            const int kk = kr + 16 * pass, k = k0 + kk;
            const char* src = static_cast<const char*>(X) + ((int64_t)k * ldx + n) * ES;
            float v[4];
            if ((ES == 4 || vec) && k < K && n + 4 <= N) {
                if (ES == 4) {
                    const f32x4 x = *reinterpret_cast<const f32x4u*>(src);
#pragma unroll
                    for (int c = 0; c < 4; ++c) v[c] = x[c];
                } else if (ES == 2) {
                    const uint2 x = *reinterpret_cast<const uint2*>(src);
                    v[0] = __uint_as_float(x.x & 0xffffu);
                    v[1] = __uint_as_float(x.x >> 16);
                    v[2] = __uint_as_float(x.y & 0xffffu);
                    v[3] = __uint_as_float(x.y >> 16);
                } else {
                    const uint32_t x = *reinterpret_cast<const uint32_t*>(src);
#pragma unroll
                    for (int c = 0; c < 4; ++c) v[c] = __uint_as_float((x >> (8 * c)) & 0xffu);
                }
            } else {
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    v[c] = 0.f;
                    if (k < K && n + c < N) {
                        if (ES == 4) v[c] = reinterpret_cast<const float*>(src)[c];
                        else if (ES == 2) v[c] = __uint_as_float(reinterpret_cast<const uint16_t*>(src)[c]);
                        else v[c] = __uint_as_float(reinterpret_cast<const uint8_t*>(src)[c]);
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) tile[kk][4 * n4 + c] = v[c];
        }
    }
    __syncthreads();
    {
        const int nn = t >> 2, kq = t & 3;  // packed row n0 + nn, k0 + 16 kq .. + 15
        const int n = n0 + nn, k = k0 + 16 * kq;
        if (n < Np && k < Kp) {
            const int64_t o = (int64_t)n * Kp + k;
            float v[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) v[j] = tile[16 * kq + j][nn];
            if (MODE == MODE_F32) {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    *reinterpret_cast<f32x4*>(static_cast<float*>(P) + o + 4 * q) =
                        f32x4{v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]};
            } else if (MODE == MODE_X3) {
                bf16x8 h[2], l[2];
                split_bf16x8(v, h[0], l[0]);
                split_bf16x8(v + 8, h[1], l[1]);
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    *reinterpret_cast<bf16x8*>(static_cast<__bf16*>(P) + o + 8 * q) = h[q];
                    *reinterpret_cast<bf16x8*>(static_cast<__bf16*>(Plo) + o + 8 * q) = l[q];
                }
            } else if (MODE == MODE_BF16) {
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    uint32_t w[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        w[e] = __float_as_uint(v[8 * q + 2 * e]) | (__float_as_uint(v[8 * q + 2 * e + 1]) << 16);
                    *reinterpret_cast<u32x4*>(static_cast<uint16_t*>(P) + o + 8 * q) = u32x4{w[0], w[1], w[2], w[3]};
                }
            } else {
                uint32_t w[4];
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    w[e] = __float_as_uint(v[4 * e]) | (__float_as_uint(v[4 * e + 1]) << 8) |
                           (__float_as_uint(v[4 * e + 2]) << 16) | (__float_as_uint(v[4 * e + 3]) << 24);
                *reinterpret_cast<u32x4*>(static_cast<uint8_t*>(P) + o) = u32x4{w[0], w[1], w[2], w[3]};
            }
        }
    }
    __syncthreads();
}

// ------------------------------------------------------------------ main loop
// MS: the MFMA block (32: 32 x 32 outputs, 16 per lane; 16: 16 x 16, 4 per lane).
template <int MODE_, int BM_, int BN_, int BK_, int WGM_, int WGN_, int NS_, int MS_ = 32>
struct PCfg {
    static constexpr int MODE = MODE_, BM = BM_, BN = BN_, BK = BK_, WGM = WGM_, WGN = WGN_;
    static constexpr int NS = NS_;  // LDS stages (panels in flight = NS - 1)
    static constexpr int MS = MS_;
    static constexpr int LG = 64 / MS;                   // lane groups along k of one MFMA
    static constexpr int AR = MS * MS / 64;              // accumulator registers per lane per block
    using Acc = typename std::conditional<MS == 32, f32x16, f32x4>::type;
    static constexpr int ES = (MODE == MODE_FP8) ? 1 : (MODE == MODE_F32) ? 4 : 2;  // bytes
    static constexpr int NT = 64 * WGM * WGN, NW = WGM * WGN;
    static constexpr int KU = 16 / ES;                   // k per 16-byte unit
    static constexpr int UK = BK / KU;                   // units per packed row per panel
    // units per lane per MFMA group: one (f32: the four 32x32x2 or 16x16x4 MFMAs
    // of its four k; bf16 and x3: 8 k) or two (e4m3: 32 k); k per group MK:
    // 32 x 32 blocks: f32 8, bf16 16, e4m3 64; 16 x 16: f32 16, bf16 32, e4m3 128
    static constexpr int UPL = (MODE == MODE_FP8) ? 2 : 1;
    static constexpr int MK = LG * UPL * KU;
    static constexpr int NG = BK / MK;
    static constexpr int WTM = BM / WGM, WTN = BN / WGN, TM = WTM / MS, TN = WTN / MS;
    // output row and column of accumulator register r of a block, for `lane`
    __device__ __forceinline__ static int out_row(int r, int lane)
    {
        return MS == 32 ? 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3) : 4 * (lane >> 4) + r;
    }
    __device__ __forceinline__ static int out_col(int lane) { return lane & (MS - 1); }
    static constexpr int NARR = (MODE == MODE_X3) ? 2 : 1;
    static constexpr int LDS_A = BM * UK * 16, LDS_B = BN * UK * 16;
    static constexpr int LDS_STAGE = NARR * (LDS_A + LDS_B);
    static constexpr int LDS_BYTES = NS * LDS_STAGE;
    // waves per SIMD the register allocation must allow: the workgroups whose
    // LDS fits in a CU's 160 KB, NW / 4 waves per SIMD each, at most four
    static constexpr int WG_PER_CU = (160 * 1024) / LDS_BYTES;
    static constexpr int WAVES_PER_EU =
        (NW / 4) * WG_PER_CU > 4 ? 4 : ((NW / 4) * WG_PER_CU < 1 ? 1 : (NW / 4) * WG_PER_CU);
    // direct-to-LDS instructions (64 units each) per wave per array per panel
    static constexpr int A_INSTR = BM * UK / 64 / NW, B_INSTR = BN * UK / 64 / NW;
    static constexpr int LOADS_PER_STAGE = NARR * (A_INSTR + B_INSTR);
    static_assert(NS >= 2 && (NS - 2) * LOADS_PER_STAGE <= 63, "vmcnt holds at most 63");
    // a panel never straddles a 128-wide K scale block
    static_assert(BK % MK == 0 && 128 % BK == 0, "panels tile K");
    static_assert((BM * UK) % (64 * NW) == 0 && (BN * UK) % (64 * NW) == 0, "loads divide among waves");
    static_assert(UK <= 16 && 16 % UK == 0, "swizzle");
    static_assert(WTM % MS == 0 && WTN % MS == 0, "whole blocks");
    static_assert(MS == 32 || MS == 16, "MFMA block");
    static_assert(LDS_BYTES <= 160 * 1024, "LDS");
};

// Physical unit of (row, logical unit u): rows of UK units, u XORed with bits
// of the row so that 16 consecutive rows at fixed u fall on 16 distinct
// 16-byte bank groups.
template <int UK>
__device__ __forceinline__ int pk_slot(int row, int u)
{
    return row * UK + (u ^ ((row / (16 / UK)) & (UK - 1)));
}

// Issue the direct-to-LDS loads of one panel for one packed array.  Wave
// instruction ig moves 64 consecutive LDS units: rows ig*(64/UK) .. of the
// tile, all UK units of each.  Lane l takes LDS unit ig*64 + l, i.e. row
// ig*(64/UK) + l/UK, physical column l%UK, which holds logical unit
// (l%UK) ^ f(row).  For the swizzle f(row) = (row / (16/UK)) & (UK-1) this is
// (l%UK) ^ (l/16) ^ ((4*ig) & (UK-1)): one per-lane byte offset (lane_off)
// XORed with a uniform constant per instruction.  The row part of the
// address is the uniform soffset, so each load costs one VGPR at most.
template <int UK, int NI>
__device__ __forceinline__ void load_panel(__amdgpu_buffer_rsrc_t rsrc, int lane_off, int row_bytes,
                                           int k_byte0, char* lds, int wave)
{
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int ig = wave * NI + i;
        const int voff = lane_off ^ (((4 * ig) & (UK - 1)) * 16);
        const int soff = ig * (64 / UK) * row_bytes + k_byte0;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            rsrc, (__attribute__((address_space(3))) void*)(lds + ig * 64 * 16), 16, voff, soff, 0, 0);
    }
}

// Buffer resource over `bytes` bytes from `base` (raw, untyped 32-bit format);
// reads beyond `bytes` return zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const char* base, int bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(base), 0, bytes, 0x00020000);
}

// s_waitcnt vmcnt(N) with expcnt and lgkmcnt left unconstrained (gfx9 encoding:
// vmcnt[3:0] in bits 3:0, vmcnt[5:4] in bits 15:14, expcnt 6:4, lgkmcnt 11:8).
template <int N>
__device__ __forceinline__ void wait_vmcnt()
{
    __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

// Workgroup barrier of the panel pipeline.  It carries no memory fence: a
// workgroup fence would make every wave wait for all of its outstanding loads
// (vmcnt(0)), including the panels issued ahead, and collapse the pipeline to
// one panel in flight.  Ordering comes from the explicit vmcnt wait before it
// (this wave's loads of the panel have reached LDS), the barrier itself (every
// wave's have), and the compiler barriers, which keep LDS reads and the next
// loads on their side of it.  The previous panel's LDS reads are complete at
// the barrier: their MFMAs, which consume them, come before it.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// This wave's LDS reads (and scalar loads) complete.
__device__ __forceinline__ void wait_lds_reads() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

struct PackedArgs {
    const char* A;    // packed A (hi), Rp_a x Kp
    const char* Alo;  // x3: packed A lo
    const char* B;    // packed B^T (hi), Rp_b x Kp
    const char* Blo;
    float* C;
    const float* sA;
    const float* sB;
    int64_t ldc, lds_a, lds_b;
    int64_t lda, ldb;  // in-place tiles: the caller's row strides (elements)
    int M, N, K, Kp;
    float alpha, beta;
    int tiles_m, tiles_n, group_m, xcd_remap;
};

// Operands of one MFMA group (MK consecutive k) for all of a wave's blocks.
template <class CF>
struct PkOps {
    static constexpr int AV = (CF::MODE == MODE_FP8) ? 2 : 1;  // 16-byte units per operand
    static constexpr int NA = (CF::MODE == MODE_X3) ? 2 : 1;   // hi (+ lo)
    u32x4 a[NA][CF::TM][AV];
    u32x4 b[NA][CF::TN][AV];
};

template <class CF>
__device__ __forceinline__ void pk_load(const char* stage, PkOps<CF>& o, int g, int wm0, int wn0,
                                        int lane)
{
    constexpr int UK = CF::UK, UPL = CF::UPL, MS = CF::MS;
    const int h = lane / MS, l32 = lane & (MS - 1);  // lane group along k, row in the block
#pragma unroll
    for (int v = 0; v < PkOps<CF>::AV; ++v) {
        const int u = (CF::LG * g + h) * UPL + v;
#pragma unroll
        for (int x = 0; x < PkOps<CF>::NA; ++x) {
            const char* la = stage + x * CF::LDS_A;
            const char* lb = stage + CF::NARR * CF::LDS_A + x * CF::LDS_B;
#pragma unroll
            for (int i = 0; i < CF::TM; ++i)
                o.a[x][i][v] = *reinterpret_cast<const u32x4*>(la + pk_slot<UK>(wm0 + MS * i + l32, u) * 16);
#pragma unroll
            for (int j = 0; j < CF::TN; ++j)
                o.b[x][j][v] = *reinterpret_cast<const u32x4*>(lb + pk_slot<UK>(wn0 + MS * j + l32, u) * 16);
        }
    }
}

// The MFMA of each form for either block size, chosen by the accumulator type
// (f32x16: 32 x 32 blocks, f32x4: 16 x 16).
__device__ __forceinline__ f32x16 mma_f32(float a, float b, f32x16 c)
{
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mma_f32(float a, float b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x16 mma_bf16(bf16x8 a, bf16x8 b, f32x16 c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mma_bf16(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
// format codes 0/0: both operands OCP e4m3; sa8, sb8: block scales (E8M0)
__device__ __forceinline__ f32x16 mma_fp8(i32x8 a, i32x8 b, f32x16 c, int sa8, int sb8)
{
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, sa8, 0, sb8);
}
__device__ __forceinline__ f32x4 mma_fp8(i32x8 a, i32x8 b, f32x4 c, int sa8, int sb8)
{
    return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, 0, sa8, 0, sb8);
}

// e4m3: sa8, sb8 are the matrix core's block scales of A and B (E8M0: byte
// e means 2^(e - 127), the same as a float32's biased exponent field), the
// same for every lane.  Constant zeros select the instruction without scales.
template <class CF>
__device__ __forceinline__ void pk_compute(const PkOps<CF>& o, typename CF::Acc (&acc)[CF::TM][CF::TN],
                                           int sa8 = 0, int sb8 = 0)
{
    if (CF::MODE == MODE_F32) {
        // element e of a lane's unit is k = 4*(LG g + lane group) + e for both
        // operands, so MFMA e pairs equal k in A and B.  (The elements are
        // copied out before the bit cast: a bit cast applied to a vector
        // element in place compiles to a read of element 0.)
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int i = 0; i < CF::TM; ++i)
#pragma unroll
                for (int j = 0; j < CF::TN; ++j) {
                    const uint32_t xa = o.a[0][i][0][e], xb = o.b[0][j][0][e];
                    acc[i][j] = mma_f32(__builtin_bit_cast(float, xa), __builtin_bit_cast(float, xb), acc[i][j]);
                }
    } else if (CF::MODE == MODE_FP8) {
#pragma unroll
        for (int i = 0; i < CF::TM; ++i)
#pragma unroll
            for (int j = 0; j < CF::TN; ++j) {
                const u32x4 a0 = o.a[0][i][0], a1 = o.a[0][i][PkOps<CF>::AV - 1];
                const u32x4 b0 = o.b[0][j][0], b1 = o.b[0][j][PkOps<CF>::AV - 1];
                const i32x8 x = {(int)a0[0], (int)a0[1], (int)a0[2], (int)a0[3],
                                 (int)a1[0], (int)a1[1], (int)a1[2], (int)a1[3]};
                const i32x8 y = {(int)b0[0], (int)b0[1], (int)b0[2], (int)b0[3],
                                 (int)b1[0], (int)b1[1], (int)b1[2], (int)b1[3]};
                acc[i][j] = mma_fp8(x, y, acc[i][j], sa8, sb8);
            }
    } else {
        if (CF::MODE == MODE_X3) {
            // small terms first: lo*hi, hi*lo, then hi*hi
#pragma unroll
            for (int i = 0; i < CF::TM; ++i)
#pragma unroll
                for (int j = 0; j < CF::TN; ++j)
                    acc[i][j] = mma_bf16(__builtin_bit_cast(bf16x8, o.a[PkOps<CF>::NA - 1][i][0]),
                                         __builtin_bit_cast(bf16x8, o.b[0][j][0]), acc[i][j]);
#pragma unroll
            for (int i = 0; i < CF::TM; ++i)
#pragma unroll
                for (int j = 0; j < CF::TN; ++j)
                    acc[i][j] = mma_bf16(__builtin_bit_cast(bf16x8, o.a[0][i][0]),
                                         __builtin_bit_cast(bf16x8, o.b[PkOps<CF>::NA - 1][j][0]), acc[i][j]);
        }
#pragma unroll
        for (int i = 0; i < CF::TM; ++i)
#pragma unroll
            for (int j = 0; j < CF::TN; ++j)
                acc[i][j] = mma_bf16(__builtin_bit_cast(bf16x8, o.a[0][i][0]),
                                     __builtin_bit_cast(bf16x8, o.b[0][j][0]), acc[i][j]);
    }
}

// Operand policy of packed_tile over the packed LDS layout: the registers of
// one MFMA group, their LDS reads and the MFMAs, and how many of each there
// are (for interleaving).
template <class CF>
struct PackedOps {
    using Ops = PkOps<CF>;
    static constexpr int NREAD = PkOps<CF>::AV * PkOps<CF>::NA * (CF::TM + CF::TN);
    static constexpr int NMFMA = CF::TM * CF::TN * (CF::MODE == MODE_X3 ? 3 : CF::MODE == MODE_F32 ? 4 : 1);
    __device__ __forceinline__ static void load(const char* stage, Ops& o, int g, int wm0, int wn0, int lane)
    {
        pk_load<CF>(stage, o, g, wm0, wn0, lane);
    }
    __device__ __forceinline__ static void compute(const Ops& o, typename CF::Acc (&acc)[CF::TM][CF::TN],
                                                   int sa8 = 0, int sb8 = 0)
    {
        pk_compute<CF>(o, acc, sa8, sb8);
    }
};

// MFMAs over one LDS stage.  Operand registers are double-buffered: the reads
// of group g + 1 are issued before the MFMAs of group g, and the scheduler is
// asked to interleave them, so LDS latency hides behind the matrix unit.
struct NoIssue {
    __device__ __forceinline__ void operator()() const {}
};

// `then` runs after the first group's LDS reads are issued (the caller issues
// the next panel's loads there, so the reads do not queue behind them);
// `before_last` runs before the last group's MFMAs, whose operands are the
// last LDS reads of the stage (the caller may refill the stage from there).
// MX: the e4m3 MFMAs take the block scales (sa8, sb8); otherwise none.
template <class CF, class OP = PackedOps<CF>, bool MX = false, class F = NoIssue, class G = NoIssue>
__device__ __forceinline__ void pk_mma(const char* stage, typename CF::Acc (&acc)[CF::TM][CF::TN], int wm0,
                                       int wn0, int lane, const F& then = F(), const G& before_last = G(),
                                       int sa8 = 0, int sb8 = 0)
{
    constexpr int NREAD = OP::NREAD;
    constexpr int NMFMA = OP::NMFMA;
    typename OP::Ops ops[2];
    OP::load(stage, ops[0], 0, wm0, wn0, lane);
    then();
#pragma unroll
    for (int g = 0; g < CF::NG; ++g) {
        if (g + 1 < CF::NG) OP::load(stage, ops[(g + 1) & 1], g + 1, wm0, wn0, lane);
        else before_last();
        if constexpr (MX) OP::compute(ops[g & 1], acc, sa8, sb8);
        else OP::compute(ops[g & 1], acc);
        if (g + 1 < CF::NG) {
            // one LDS read between consecutive MFMAs while both last
#pragma unroll
            for (int k = 0; k < (NREAD < NMFMA ? NREAD : NMFMA); ++k) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // DS read
            }
        }
    }
}

// Scales of A's and B's tiles for block (row0, col0) and K scale block kb.
// (The loads are vector loads, counted by vmcnt like the panel loads:
// packed_tile issues them one panel ahead of their use.)
__device__ __forceinline__ void block_scales(const PackedArgs& a, int row0, int col0, int kb, float& sa,
                                             float& sb)
{
    if (row0 >= a.M || col0 >= a.N) {  // a block of padding: never stored
        sa = sb = 1.f;
        return;
    }
    const int64_t ia = __builtin_amdgcn_readfirstlane((int)((row0 / 128) * a.lds_a + kb));
    const int64_t ib = __builtin_amdgcn_readfirstlane((int)(kb * a.lds_b + col0 / 128));
    sa = a.sA[ia];
    sb = a.sB[ib];
}
__device__ __forceinline__ float block_scale(const PackedArgs& a, int row0, int col0, int kb)
{
    float sa, sb;
    block_scales(a, row0, col0, kb, sa, sb);
    return sa * sb;
}

// A float32 scale s as 2^(e8 - 127) * m with e8 its biased exponent (the E8M0
// byte the e4m3 matrix core applies exactly) and m in [1, 2) (sign kept);
// zero, subnormal and non-finite s keep everything in m (e8 = 127: 2^0).
__device__ __forceinline__ void split_scale(float s, int& e8, float& m)
{
    const uint32_t u = __float_as_uint(s), ex = (u >> 23) & 0xffu;
    if (ex == 0u || ex == 0xffu) {
        e8 = 127;
        m = s;
    } else {
        e8 = (int)ex;
        m = __uint_as_float((u & 0x807fffffu) | (127u << 23));
    }
}

// A-side panel loads over packed rows of A (a.A, and a.Alo for x3): the
// default operand source of packed_tile.
template <class CF>
struct PackedRowsA {
    struct Geom {};
    static constexpr int LOADS = CF::NARR * CF::A_INSTR;  // loads per wave per panel
    __amdgpu_buffer_rsrc_t r, rl;
    int lane_off, row_bytes, wave;

    __device__ __forceinline__ void init(const PackedArgs& a, int m0, int lane, int wave_, const Geom&)
    {
        wave = wave_;
        row_bytes = a.Kp * CF::ES;
        r = make_rsrc(a.A + (int64_t)m0 * row_bytes, CF::BM * row_bytes);
        rl = r;
        if (CF::MODE == MODE_X3) rl = make_rsrc(a.Alo + (int64_t)m0 * row_bytes, CF::BM * row_bytes);
        lane_off = (lane / CF::UK) * row_bytes + (((lane % CF::UK) ^ (lane / 16)) & (CF::UK - 1)) * 16;
    }

    __device__ __forceinline__ void issue(int panel, char* stage) const
    {
        const int kb = panel * CF::BK * CF::ES;
        load_panel<CF::UK, CF::A_INSTR>(r, lane_off, row_bytes, kb, stage, wave);
        if (CF::MODE == MODE_X3)
            load_panel<CF::UK, CF::A_INSTR>(rl, lane_off, row_bytes, kb, stage + CF::LDS_A, wave);
    }
};

// B-side panel loads over packed rows of B^T (a.B, and a.Blo for x3): the
// default operand source of packed_tile.  `stage` is the B part of an LDS stage.
template <class CF>
struct PackedRowsB {
    static constexpr int LOADS = CF::NARR * CF::B_INSTR;
    __amdgpu_buffer_rsrc_t r, rl;
    int lane_off, row_bytes, wave;

    __device__ __forceinline__ void init(const PackedArgs& a, int n0, int lane, int wave_)
    {
        wave = wave_;
        row_bytes = a.Kp * CF::ES;
        r = make_rsrc(a.B + (int64_t)n0 * row_bytes, CF::BN * row_bytes);
        rl = r;
        if (CF::MODE == MODE_X3) rl = make_rsrc(a.Blo + (int64_t)n0 * row_bytes, CF::BN * row_bytes);
        lane_off = (lane / CF::UK) * row_bytes + (((lane % CF::UK) ^ (lane / 16)) & (CF::UK - 1)) * 16;
    }

    __device__ __forceinline__ void issue(int panel, char* stage) const
    {
        const int kb = panel * CF::BK * CF::ES;
        load_panel<CF::UK, CF::B_INSTR>(r, lane_off, row_bytes, kb, stage, wave);
        if (CF::MODE == MODE_X3)
            load_panel<CF::UK, CF::B_INSTR>(rl, lane_off, row_bytes, kb, stage + CF::LDS_B, wave);
    }
};

// Epilogue of a whole tile: C = alpha * scale * acc (+ beta * C), predicated
// only on partial tiles.  sc(i, j) is the scale product that multiplies the
// sums of block (i, j) (1 for unscaled forms).
template <class CF>
struct TileStore {
    const PackedArgs& a;
    int m0, n0;
    template <class SC>
    __device__ __forceinline__ void operator()(typename CF::Acc (&acc)[CF::TM][CF::TN], const SC& sc, int wm0,
                                               int wn0, int lane) const
    {
        // the addresses below are computed here, not hoisted out of a loop over
        // tiles where they would hold registers through the main loop
        asm volatile("" : "+v"(lane));
        write_c<CF::TM, CF::TN, CF::AR>(
            a.C, a.ldc, a.M, a.N, a.beta, CF::out_row(0, lane), CF::out_col(lane),
            [&](int i, int j, float (&v)[CF::AR]) {
                const float f = a.alpha * sc(i, j);
#pragma unroll
                for (int r = 0; r < CF::AR; ++r) v[r] = f * acc[i][j][r];
            },
            [&](int i, int j, int& r0, int& c0) {
                r0 = m0 + wm0 + CF::MS * i;
                c0 = n0 + wn0 + CF::MS * j;
            },
            [](int r) { return CF::out_row(r, 0); });
    }
};

// Panels [p0, p0 + np) of one BM x BN macro-tile at (m0, n0) of problem `a`;
// `lds` holds CF::LDS_BYTES.  AL and BL bring the A and B panels into an LDS
// stage (A first, B at offset NARR * LDS_A), each issuing a fixed number of
// loads per wave per panel (AL::LOADS + BL::LOADS in all); OP reads the MFMA
// operands from a stage and runs the MFMAs; EPI receives the sums (see
// TileStore).  By default both operands come from packed rows (of A and of
// B^T), which must extend to m0 + BM and n0 + BN, and K to a multiple of BK,
// with zeros beyond K.  The caller separates consecutive calls that reuse
// `lds` with a barrier.
// SCALED: a.sA and a.sB hold per-tile scales (bf16 and e4m3 only; the caller
// branches on a.sA once, so each loop is compiled for one case).
template <class CF, class AL, class BL, class OP, bool SCALED, class EPI>
__device__ __forceinline__ void packed_tile_range(const PackedArgs& a, int m0, int n0, char* lds,
                                                  const typename AL::Geom& geom, int p0, int np,
                                                  const EPI& epi)
{
    const int t = threadIdx.x, lane = t & 63;
    // the wave index is uniform; readfirstlane lets the compiler keep it (and the
    // load offsets and LDS bases derived from it) in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int wm0 = (wave / CF::WGN) * CF::WTM, wn0 = (wave % CF::WGN) * CF::WTN;
    AL al;
    al.init(a, m0, lane, wave, geom);
    BL bl;
    bl.init(a, n0, lane, wave);
    constexpr bool scaled = SCALED && (CF::MODE == MODE_BF16 || CF::MODE == MODE_FP8);

    typename CF::Acc acc[CF::TM][CF::TN];
#pragma unroll
    for (int i = 0; i < CF::TM; ++i)
#pragma unroll
        for (int j = 0; j < CF::TN; ++j)
#pragma unroll
            for (int r = 0; r < CF::AR; ++r) acc[i][j][r] = 0.f;

    const int npanel = np;
    auto issue = [&](int panel, char* stage) {  // panel: index within the range
        al.issue(p0 + panel, stage);
        bl.issue(p0 + panel, stage + CF::NARR * CF::LDS_A);
    };

    // Scaled forms: acc is kept divided by the scale product of the current K
    // block (128 deep).  The products of the next block are loaded one panel
    // ahead, before that panel's successor is issued, so the waits of the panel
    // pipeline cover them; loading them where they are used would drain the
    // panels in flight at every block boundary.  (They are vector loads: C is
    // written by the same kernel and may alias the scales.)
    // A wave tile no larger than a 128 x 128 scale tile lies inside one (tiles
    // start at multiples of their size), so one product serves all its blocks.
    constexpr bool one_scale = CF::WTM <= 128 && CF::WTN <= 128;
    constexpr int SM = one_scale ? 1 : CF::TM, SN = one_scale ? 1 : CF::TN;
    // e4m3 with one product per wave: the powers of two of sA and sB go to the
    // matrix core as its block scales (e8a, e8b), and acc is kept in units of
    // the product of their mantissas, m = fl32(ma * mb) = fl32(sA * sB) / 2^E;
    // with power-of-two scales m stays 1 and acc is never rescaled.
    constexpr bool mx = scaled && one_scale && CF::MODE == MODE_FP8;
    int kb_cur = (p0 * CF::BK) / 128;
    float sc_cur[SM][SN], sc_next[SM][SN];  // mx: sc_cur holds m, sc_next the raw sB
    int e8a = 127, e8b = 127;
    float sa_next = 1.f;
    auto load_scales = [&](int kb, float (&dst)[SM][SN]) {
        if constexpr (mx) {
            block_scales(a, m0 + wm0, n0 + wn0, kb, sa_next, dst[0][0]);
        } else {
#pragma unroll
            for (int i = 0; i < SM; ++i)
#pragma unroll
                for (int j = 0; j < SN; ++j)
                    dst[i][j] = block_scale(a, m0 + wm0 + CF::MS * i, n0 + wn0 + CF::MS * j, kb);
        }
    };
    // the unit of the block whose raw scales are sa_next and sc_next (mx)
    auto mx_unit = [&](int& ea, int& eb) {
        float ma, mb;
        split_scale(sa_next, ea, ma);
        split_scale(sc_next[0][0], eb, mb);
        return ma * mb;
    };
    // issued before the first panels, so the first panel's wait covers them
    if constexpr (scaled) {
        if constexpr (mx) {
            load_scales(kb_cur, sc_next);
        } else {
            load_scales(kb_cur, sc_cur);
        }
    }

    // Pipeline: panels p go to stage p % NS; NS - 1 panels are in flight.
    constexpr int NS = CF::NS, L = AL::LOADS + BL::LOADS;
    static_assert((NS - 2) * L <= 63, "vmcnt holds at most 63");
    for (int p = 0; p < NS - 1 && p < npanel; ++p) issue(p, lds + p * CF::LDS_STAGE);
    bool first_block = true;  // mx: the unit of the first block is set at its first panel
    auto prefetch = [&](int s) {  // during panel s: the scales of panel s + 1 if it opens a block
        if (!scaled || s + 1 >= npanel) return;
        const int kb = ((p0 + s + 1) * CF::BK) / 128;
        if (kb != ((p0 + s) * CF::BK) / 128) load_scales(kb, sc_next);
    };
    // new K scale block at panel s: move acc to the new block's scale product
    auto rescale = [&](int s) {
        if (!scaled) return;
        const int kb = ((p0 + s) * CF::BK) / 128;
        if constexpr (mx) {
            if (first_block) {
                first_block = false;
                sc_cur[0][0] = mx_unit(e8a, e8b);
                return;
            }
            if (kb == kb_cur) return;
            const float m = mx_unit(e8a, e8b);
            const float ratio = sc_cur[0][0] / m;
            if (ratio != 1.f) {
#pragma unroll
                for (int i = 0; i < CF::TM; ++i)
#pragma unroll
                    for (int j = 0; j < CF::TN; ++j)
#pragma unroll
                        for (int r = 0; r < CF::AR; ++r) acc[i][j][r] *= ratio;
            }
            sc_cur[0][0] = m;
            kb_cur = kb;
            return;
        }
        if (s == 0 || kb == kb_cur) return;
        if constexpr (one_scale) {
            // one product per wave: nothing to do when it does not change (acc * 1 == acc)
            const float ratio = sc_cur[0][0] / sc_next[0][0];
            if (ratio != 1.f) {
#pragma unroll
                for (int i = 0; i < CF::TM; ++i)
#pragma unroll
                    for (int j = 0; j < CF::TN; ++j)
#pragma unroll
                        for (int r = 0; r < CF::AR; ++r) acc[i][j][r] *= ratio;
            }
        } else {
#pragma unroll
            for (int i = 0; i < CF::TM; ++i)
#pragma unroll
                for (int j = 0; j < CF::TN; ++j) {
                    const float ratio = sc_cur[i][j] / sc_next[i][j];
#pragma unroll
                    for (int r = 0; r < CF::AR; ++r) acc[i][j][r] *= ratio;
                }
        }
#pragma unroll
        for (int i = 0; i < SM; ++i)
#pragma unroll
            for (int j = 0; j < SN; ++j) sc_cur[i][j] = sc_next[i][j];
        kb_cur = kb;
    };
    if constexpr (NS == 2 && (CF::MODE == MODE_FP8 || (CF::NG == 1 && CF::BM >= 128))) {
        // Two stages, refilled early: panel s + 2 goes into panel s's stage as
        // soon as every wave holds the operands of its last group of panel s (a
        // barrier before that group's MFMAs), so its loads have the rest of panel
        // s and all of panel s + 1 to land, at one more barrier per panel.
        // Measured on MI355X: e4m3 +4-6%, one-group panels of 128-row tiles (x3
        // 128x128x16) twice as fast; bf16 with four groups per panel 11% slower
        // and the 64 x 64 in-place x3 tiles of the grouped launch about 5%, so
        // the others keep the loop below.
        static_assert(L <= 63, "vmcnt holds at most 63");
        if (1 < npanel) issue(1, lds + CF::LDS_STAGE);
        for (int s = 0; s < npanel; ++s) {
            // this wave's loads of panel s have landed once at most those of panel
            // s + 1 remain (issued after them); the barrier covers every wave's
            if (s + 1 < npanel) wait_vmcnt<L>();
            else wait_vmcnt<0>();
            lds_barrier();
            rescale(s);   // consumes the scales prefetched during panel s - 1 ...
            prefetch(s);  // ... before they are replaced by those of panel s + 1
            char* stage = lds + (s % NS) * CF::LDS_STAGE;
            pk_mma<CF, OP, mx>(stage, acc, wm0, wn0, lane, NoIssue(), [&] {
                wait_lds_reads();  // this wave's reads of the stage are done ...
                lds_barrier();     // ... and every wave's: the stage is free
                if (s + 2 < npanel) issue(s + 2, stage);
            }, e8a, e8b);
        }
    } else if constexpr (NS == 2) {
        for (int s = 0; s < npanel; ++s) {
            // this wave's loads of panel s have landed once at most the loads of the
            // panels issued after it remain; then the barrier covers every wave's loads
            // and frees the stage that panel s - 1 occupied
            if (s + NS - 2 < npanel) wait_vmcnt<(NS - 2) * L>();
            else wait_vmcnt<0>();
            lds_barrier();
            rescale(s);   // consumes the scales prefetched during panel s - 1 ...
            prefetch(s);  // ... before they are replaced by those of panel s + 1
            // On 256 x 256 tiles the next panel's loads go out after the first group of
            // LDS reads, which then do not wait behind them; on smaller tiles, with
            // fewer MFMAs per panel to cover the loads, they go out first.
            auto next = [&] {
                if (s + NS - 1 < npanel) issue(s + NS - 1, lds + ((s + NS - 1) % NS) * CF::LDS_STAGE);
            };
            if constexpr (CF::BM >= 256 && CF::BN >= 256) {
                pk_mma<CF, OP, mx>(lds + (s % NS) * CF::LDS_STAGE, acc, wm0, wn0, lane, next, NoIssue(), e8a, e8b);
            } else {
                next();
                pk_mma<CF, OP, mx>(lds + (s % NS) * CF::LDS_STAGE, acc, wm0, wn0, lane, NoIssue(), NoIssue(), e8a,
                                   e8b);
            }
        }
    } else {
        // Three or more stages: the next panel has landed before this one ends, so
        // the first group of its operands is read from LDS while the last group of
        // this panel runs on the MFMAs; neither the barrier nor the LDS latency of a
        // panel boundary leaves the matrix cores idle.  The barrier that admits
        // panel s + 1 follows this wave's last LDS read of panel s, so the refill of
        // panel s's stage (issued after it, at the top of the next iteration) never
        // overtakes a read.
        constexpr int NPAIR = OP::NREAD < OP::NMFMA ? OP::NREAD : OP::NMFMA;
        typename OP::Ops ops[2];
        if (NS - 2 < npanel) wait_vmcnt<(NS - 2) * L>();
        else wait_vmcnt<0>();
        lds_barrier();
        OP::load(lds, ops[0], 0, wm0, wn0, lane);
        for (int s = 0; s < npanel; ++s) {
            rescale(s);
            prefetch(s);
            if (s + NS - 1 < npanel) issue(s + NS - 1, lds + ((s + NS - 1) % NS) * CF::LDS_STAGE);
            const char* stage = lds + (s % NS) * CF::LDS_STAGE;
#pragma unroll
            for (int g = 0; g < CF::NG; ++g) {
                bool read = false;
                if (g + 1 < CF::NG) {
                    OP::load(stage, ops[(g + 1) & 1], g + 1, wm0, wn0, lane);
                    read = true;
                } else if (s + 1 < npanel) {
                    if (s + NS - 1 < npanel) wait_vmcnt<(NS - 2) * L>();
                    else wait_vmcnt<0>();
                    wait_lds_reads();
                    lds_barrier();
                    OP::load(lds + ((s + 1) % NS) * CF::LDS_STAGE, ops[CF::NG & 1], 0, wm0, wn0, lane);
                    read = true;
                }
                if constexpr (mx) OP::compute(ops[g & 1], acc, e8a, e8b);
                else OP::compute(ops[g & 1], acc);
                if (read) {
#pragma unroll
                    for (int k = 0; k < NPAIR; ++k) {
                        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
                        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // DS read
                    }
                }
            }
            if (CF::NG & 1) ops[0] = ops[1];  // the next panel's first group
        }
    }

    epi(acc, [&](int i, int j) { return scaled ? sc_cur[i % SM][j % SN] : 1.f; }, wm0, wn0, lane);
}

// One whole macro-tile (all K panels) with the standard epilogue.
template <class CF, class AL = PackedRowsA<CF>, class BL = PackedRowsB<CF>, class OP = PackedOps<CF>>
__device__ __forceinline__ void packed_tile(const PackedArgs& a, int m0, int n0, char* lds,
                                            const typename AL::Geom& geom = typename AL::Geom())
{
    const int np = (a.K + CF::BK - 1) / CF::BK;
    if ((CF::MODE == MODE_BF16 || CF::MODE == MODE_FP8) && a.sA)
        packed_tile_range<CF, AL, BL, OP, true>(a, m0, n0, lds, geom, 0, np, TileStore<CF>{a, m0, n0});
    else
        packed_tile_range<CF, AL, BL, OP, false>(a, m0, n0, lds, geom, 0, np, TileStore<CF>{a, m0, n0});
}

}  // namespace tg
