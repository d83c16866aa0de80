// Packed-operand gemm for every MFMA form: f32, split-bf16x3, and bf16 and
// e4m3 with per-tile scales.
//
// Array packing (Tiramisu paper, Section I, after Goto and van de Geijn) as a
// pre-pass: A (M x K, row-major) and B (K x N, row-major) are copied once into
// packed buffers whose rows are K-contiguous, in the element type the MFMA
// reads, zero-padded to multiples of kPackRows rows and kPackK columns:
//   Ap[m][k]  = conv(A[m][k]),   Bp[n][k] = conv(B[k][n])   (B transposed)
// where conv is the x3 split (two arrays, hi and lo) or a plain copy of the
// values (f32) or codes (bf16, e4m3).
// The padding turns every tile into a full tile for the loads, so the main
// kernel's K loop carries no predicates; the full/partial distinction of
// Section V-C remains only in the epilogue (masked stores for edge tiles).
//
// Main kernel: one workgroup per BM x BN macro-tile, WGM x WGN waves, each
// wave a register tile of 32x32 MFMA blocks.  K panels of BK go from the
// packed buffers straight into LDS with global_load_lds_dwordx4 (16 bytes per
// lane, no register staging), two stages, one barrier per panel: the loads of
// panel k+1 are in flight while the MFMAs consume panel k.  LDS rows hold the
// panel's KU-element units of one packed row, XOR-swizzled so that the MFMA
// operand reads of 16 consecutive rows hit distinct banks.
//
// Scaled forms: the running sum is kept divided by the current K block's scale
// product and rescaled when the K block changes, so no second accumulator set
// is needed:  acc <- acc * (s_prev / s_cur) at each 128-wide K block,
// C = alpha * s_last * acc.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <utility>

#include "../../include/tgemm.h"
#include "kargs.h"
#include "registry.h"
#include "tile_f32x3.h"

namespace tg {

constexpr int kPackRows = 256;  // packed row counts are multiples of this
constexpr int kPackK = 128;     // packed K is a multiple of this (elements)

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

// ------------------------------------------------------------------ packing
// A-side: rows of X (R x K, row stride ldx) -> P (Rp x Kp), 8 consecutive
// k per thread.  x3: X is float, P / Plo receive the bf16 hi and lo parts.
// f32: floats, copied.  bf16 / e4m3: X holds codes of ES bytes, copied.
template <int MODE>
__global__ void pack_rows_kernel(const void* X, int64_t ldx, int R, int K, void* P, void* Plo,
                                 int Rp, int Kp)
{
    const int64_t groups = (int64_t)Rp * (Kp / 8);
    for (int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gi < groups;
         gi += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(gi / (Kp / 8));
        const int k0 = (int)(gi % (Kp / 8)) * 8;
        if (MODE == MODE_F32) {
            f32x4 v0, v1;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const float v = (r < R && k0 + e < K)
                                    ? static_cast<const float*>(X)[(int64_t)r * ldx + k0 + e] : 0.f;
                if (e < 4) v0[e] = v;
                else v1[e - 4] = v;
            }
            float* dst = static_cast<float*>(P) + (int64_t)r * Kp + k0;
            *reinterpret_cast<f32x4*>(dst) = v0;
            *reinterpret_cast<f32x4*>(dst + 4) = v1;
        } else if (MODE == MODE_X3) {
            bf16x8 h, l;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                float v = 0.f;
                if (r < R && k0 + e < K) v = static_cast<const float*>(X)[(int64_t)r * ldx + k0 + e];
                __bf16 hh, ll;
                split_bf16(v, hh, ll);
                h[e] = hh;
                l[e] = ll;
            }
            *reinterpret_cast<bf16x8*>(static_cast<__bf16*>(P) + (int64_t)r * Kp + k0) = h;
            *reinterpret_cast<bf16x8*>(static_cast<__bf16*>(Plo) + (int64_t)r * Kp + k0) = l;
        } else if (MODE == MODE_BF16) {
            uint16_t w[8];
#pragma unroll
            for (int e = 0; e < 8; ++e)
                w[e] = (r < R && k0 + e < K)
                           ? static_cast<const uint16_t*>(X)[(int64_t)r * ldx + k0 + e] : (uint16_t)0;
            uint16_t* dst = static_cast<uint16_t*>(P) + (int64_t)r * Kp + k0;
            *reinterpret_cast<u32x4*>(dst) = u32x4{w[0] | ((uint32_t)w[1] << 16),
                                                   w[2] | ((uint32_t)w[3] << 16),
                                                   w[4] | ((uint32_t)w[5] << 16),
                                                   w[6] | ((uint32_t)w[7] << 16)};
        } else {
            uint32_t w0 = 0, w1 = 0;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const uint32_t v = (r < R && k0 + e < K)
                                       ? static_cast<const uint8_t*>(X)[(int64_t)r * ldx + k0 + e] : 0u;
                if (e < 4) w0 |= v << (8 * e);
                else w1 |= v << (8 * (e - 4));
            }
            uint8_t* dst = static_cast<uint8_t*>(P) + (int64_t)r * Kp + k0;
            *reinterpret_cast<uint2*>(dst) = make_uint2(w0, w1);
        }
    }
}

// B-side: X (K x N, row stride ldx) -> P (Np x Kp) = X^T, through a 64 x 64
// LDS tile (reads coalesced along N, writes coalesced along K).
template <int MODE>
__global__ void __launch_bounds__(256) pack_cols_kernel(const void* X, int64_t ldx, int K, int N,
                                                        void* P, void* Plo, int Np, int Kp)
{
    __shared__ float tile[64][65];  // x3: float values; codes: widened to 32 bits
    const int n0 = blockIdx.x * 64, k0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4
    for (int kk = ty; kk < 64; kk += 4) {
        const int k = k0 + kk, n = n0 + tx;
        float v = 0.f;
        if (k < K && n < N) {
            if (MODE == MODE_X3 || MODE == MODE_F32) v = static_cast<const float*>(X)[(int64_t)k * ldx + n];
            else if (MODE == MODE_BF16)
                v = __uint_as_float(static_cast<const uint16_t*>(X)[(int64_t)k * ldx + n]);
            else v = __uint_as_float(static_cast<const uint8_t*>(X)[(int64_t)k * ldx + n]);
        }
        tile[kk][tx] = v;
    }
    __syncthreads();
    for (int nn = ty; nn < 64; nn += 4) {
        const int n = n0 + nn, k = k0 + tx;
        if (n >= Np || k >= Kp) continue;
        const float v = tile[tx][nn];
        const int64_t o = (int64_t)n * Kp + k;
        if (MODE == MODE_F32) {
            static_cast<float*>(P)[o] = v;
        } else if (MODE == MODE_X3) {
            __bf16 hh, ll;
            split_bf16(v, hh, ll);
            static_cast<__bf16*>(P)[o] = hh;
            static_cast<__bf16*>(Plo)[o] = ll;
        } else if (MODE == MODE_BF16) {
            static_cast<uint16_t*>(P)[o] = (uint16_t)__float_as_uint(v);
        } else {
            static_cast<uint8_t*>(P)[o] = (uint8_t)__float_as_uint(v);
        }
    }
}

// ------------------------------------------------------------------ main kernel
template <int MODE_, int BM_, int BN_, int BK_, int WGM_, int WGN_, int NS_>
struct PCfg {
    static constexpr int MODE = MODE_, BM = BM_, BN = BN_, BK = BK_, WGM = WGM_, WGN = WGN_;
    static constexpr int NS = NS_;  // LDS stages (panels in flight = NS - 1)
    // waves per SIMD the register allocation must allow: two workgroups per CU
    // when one workgroup's LDS fits in half of the 160 KB
    static constexpr int ES = (MODE == MODE_FP8) ? 1 : (MODE == MODE_F32) ? 4 : 2;  // bytes
    static constexpr int WAVES_PER_EU =
        (NS_ * (MODE_ == MODE_X3 ? 2 : 1) * (BM_ + BN_) * BK_ * ES <= 80 * 1024 && WGM_ * WGN_ == 4) ? 2 : 1;
    static constexpr int NT = 64 * WGM * WGN, NW = WGM * WGN;
    static constexpr int KU = 16 / ES;                   // k per 16-byte unit
    static constexpr int UK = BK / KU;                   // units per packed row per panel
    // k per MFMA group: 32x32x64 e4m3, 32x32x16 bf16; f32 runs the four
    // 32x32x2 MFMAs of one unit per lane as a group of 8 k
    static constexpr int MK = (MODE == MODE_FP8) ? 64 : (MODE == MODE_F32) ? 8 : 16;
    static constexpr int UPL = MK / KU / 2;              // units per lane per group
    static constexpr int NG = BK / MK;
    static constexpr int WTM = BM / WGM, WTN = BN / WGN, TM = WTM / 32, TN = WTN / 32;
    static constexpr int NARR = (MODE == MODE_X3) ? 2 : 1;
    static constexpr int LDS_A = BM * UK * 16, LDS_B = BN * UK * 16;
    static constexpr int LDS_STAGE = NARR * (LDS_A + LDS_B);
    static constexpr int LDS_BYTES = NS * LDS_STAGE;
    // direct-to-LDS instructions (64 units each) per wave per array per panel
    static constexpr int A_INSTR = BM * UK / 64 / NW, B_INSTR = BN * UK / 64 / NW;
    static constexpr int LOADS_PER_STAGE = NARR * (A_INSTR + B_INSTR);
    static_assert(NS >= 2 && (NS - 2) * LOADS_PER_STAGE <= 63, "vmcnt holds at most 63");
    static_assert(BK % MK == 0 && kPackK % BK == 0 && 128 % BK == 0, "panels tile K");
    static_assert(BM <= kPackRows && BN <= kPackRows && kPackRows % BM == 0 && kPackRows % BN == 0,
                  "tiles divide the packed row padding");
    static_assert((BM * UK) % (64 * NW) == 0 && (BN * UK) % (64 * NW) == 0, "loads divide among waves");
    static_assert(UK <= 16 && 16 % UK == 0, "swizzle");
    static_assert(WTM % 32 == 0 && WTN % 32 == 0, "whole blocks");
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

struct PackedArgs {
    const char* A;    // packed A (hi), Rp_a x Kp
    const char* Alo;  // x3: packed A lo
    const char* B;    // packed B^T (hi), Rp_b x Kp
    const char* Blo;
    float* C;
    const float* sA;
    const float* sB;
    int64_t ldc, lds_a, lds_b;
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
    constexpr int UK = CF::UK, UPL = CF::UPL;
    const int h = lane >> 5, l32 = lane & 31;
#pragma unroll
    for (int v = 0; v < PkOps<CF>::AV; ++v) {
        const int u = (2 * g + h) * UPL + v;
#pragma unroll
        for (int x = 0; x < PkOps<CF>::NA; ++x) {
            const char* la = stage + x * CF::LDS_A;
            const char* lb = stage + CF::NARR * CF::LDS_A + x * CF::LDS_B;
#pragma unroll
            for (int i = 0; i < CF::TM; ++i)
                o.a[x][i][v] = *reinterpret_cast<const u32x4*>(la + pk_slot<UK>(wm0 + 32 * i + l32, u) * 16);
#pragma unroll
            for (int j = 0; j < CF::TN; ++j)
                o.b[x][j][v] = *reinterpret_cast<const u32x4*>(lb + pk_slot<UK>(wn0 + 32 * j + l32, u) * 16);
        }
    }
}

template <class CF>
__device__ __forceinline__ void pk_compute(const PkOps<CF>& o, f32x16 (&acc)[CF::TM][CF::TN])
{
    if (CF::MODE == MODE_F32) {
        // element e of a lane's unit is k = 4*(2g + lane/32) + e for both
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
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(
                        __builtin_bit_cast(float, xa), __builtin_bit_cast(float, xb), acc[i][j], 0, 0, 0);
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
                // format codes 0/0: both operands OCP e4m3; no block scaling
                acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(x, y, acc[i][j], 0, 0, 0, 0, 0, 0);
            }
    } else {
        if (CF::MODE == MODE_X3) {
            // small terms first: lo*hi, hi*lo, then hi*hi
#pragma unroll
            for (int i = 0; i < CF::TM; ++i)
#pragma unroll
                for (int j = 0; j < CF::TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                        __builtin_bit_cast(bf16x8, o.a[PkOps<CF>::NA - 1][i][0]),
                        __builtin_bit_cast(bf16x8, o.b[0][j][0]), acc[i][j], 0, 0, 0);
#pragma unroll
            for (int i = 0; i < CF::TM; ++i)
#pragma unroll
                for (int j = 0; j < CF::TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                        __builtin_bit_cast(bf16x8, o.a[0][i][0]),
                        __builtin_bit_cast(bf16x8, o.b[PkOps<CF>::NA - 1][j][0]), acc[i][j], 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < CF::TM; ++i)
#pragma unroll
            for (int j = 0; j < CF::TN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                    __builtin_bit_cast(bf16x8, o.a[0][i][0]), __builtin_bit_cast(bf16x8, o.b[0][j][0]),
                    acc[i][j], 0, 0, 0);
    }
}

// MFMAs over one LDS stage.  Operand registers are double-buffered: the reads
// of group g + 1 are issued before the MFMAs of group g, and the scheduler is
// asked to interleave them, so LDS latency hides behind the matrix unit.
template <class CF>
__device__ __forceinline__ void pk_mma(const char* stage, f32x16 (&acc)[CF::TM][CF::TN], int wm0,
                                       int wn0, int lane)
{
    constexpr int NREAD = PkOps<CF>::AV * PkOps<CF>::NA * (CF::TM + CF::TN);
    constexpr int NMFMA = CF::TM * CF::TN * (CF::MODE == MODE_X3 ? 3 : CF::MODE == MODE_F32 ? 4 : 1);
    PkOps<CF> ops[2];
    pk_load<CF>(stage, ops[0], 0, wm0, wn0, lane);
#pragma unroll
    for (int g = 0; g < CF::NG; ++g) {
        if (g + 1 < CF::NG) pk_load<CF>(stage, ops[(g + 1) & 1], g + 1, wm0, wn0, lane);
        pk_compute<CF>(ops[g & 1], acc);
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

// Scale product of block (row0, col0) for K scale block kb.
// (row0, col0 and kb are wave-uniform, so the two loads are scalar loads and do
// not count against vmcnt, which tracks the panel pipeline.)
__device__ __forceinline__ float block_scale(const PackedArgs& a, int row0, int col0, int kb)
{
    if (row0 >= a.M || col0 >= a.N) return 1.f;  // a block of padding: never stored
    const int64_t ia = __builtin_amdgcn_readfirstlane((int)((row0 / 128) * a.lds_a + kb));
    const int64_t ib = __builtin_amdgcn_readfirstlane((int)(kb * a.lds_b + col0 / 128));
    return a.sA[ia] * a.sB[ib];
}

template <class CF>
__global__ void __launch_bounds__(CF::NT, CF::WAVES_PER_EU) packed_kernel(PackedArgs a)
{
    __shared__ __attribute__((aligned(1024))) char lds[CF::LDS_BYTES];
    const TileCoord tc = map_tile(blockIdx.x, a.tiles_m, a.tiles_n, a.group_m, a.xcd_remap);
    const int m0 = tc.tm * CF::BM, n0 = tc.tn * CF::BN;
    const int t = threadIdx.x, lane = t & 63;
    // the wave index is uniform; readfirstlane lets the compiler keep it (and the
    // load offsets and LDS bases derived from it) in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int wm0 = (wave / CF::WGN) * CF::WTM, wn0 = (wave % CF::WGN) * CF::WTN;
    const int row_bytes = a.Kp * CF::ES;
    const __amdgpu_buffer_rsrc_t rA = make_rsrc(a.A + (int64_t)m0 * row_bytes, CF::BM * row_bytes);
    const __amdgpu_buffer_rsrc_t rB = make_rsrc(a.B + (int64_t)n0 * row_bytes, CF::BN * row_bytes);
    __amdgpu_buffer_rsrc_t rAl = rA, rBl = rB;
    if (CF::MODE == MODE_X3) {
        rAl = make_rsrc(a.Alo + (int64_t)m0 * row_bytes, CF::BM * row_bytes);
        rBl = make_rsrc(a.Blo + (int64_t)n0 * row_bytes, CF::BN * row_bytes);
    }
    const int lane_off = (lane / CF::UK) * row_bytes + (((lane % CF::UK) ^ (lane / 16)) & (CF::UK - 1)) * 16;
    const bool scaled = (CF::MODE == MODE_BF16 || CF::MODE == MODE_FP8) && a.sA;

    f32x16 acc[CF::TM][CF::TN];
#pragma unroll
    for (int i = 0; i < CF::TM; ++i)
#pragma unroll
        for (int j = 0; j < CF::TN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    const int npanel = (a.K + CF::BK - 1) / CF::BK;
    auto issue = [&](int panel, char* stage) {
        const int kb = panel * CF::BK * CF::ES;
        load_panel<CF::UK, CF::A_INSTR>(rA, lane_off, row_bytes, kb, stage, wave);
        if (CF::MODE == MODE_X3)
            load_panel<CF::UK, CF::A_INSTR>(rAl, lane_off, row_bytes, kb, stage + CF::LDS_A, wave);
        char* sb = stage + CF::NARR * CF::LDS_A;
        load_panel<CF::UK, CF::B_INSTR>(rB, lane_off, row_bytes, kb, sb, wave);
        if (CF::MODE == MODE_X3)
            load_panel<CF::UK, CF::B_INSTR>(rBl, lane_off, row_bytes, kb, sb + CF::LDS_B, wave);
    };

    // Pipeline: panels p go to stage p % NS; NS - 1 panels are in flight.
    constexpr int NS = CF::NS;
    for (int p = 0; p < NS - 1 && p < npanel; ++p) issue(p, lds + p * CF::LDS_STAGE);
    int kb_cur = 0;
    for (int s = 0; s < npanel; ++s) {
        // this wave's loads of panel s have landed once at most the loads of the
        // panels issued after it remain; then the barrier covers every wave's loads
        // and frees the stage that panel s - 1 occupied
        if (s + NS - 2 < npanel) wait_vmcnt<(NS - 2) * CF::LOADS_PER_STAGE>();
        else wait_vmcnt<0>();
        __syncthreads();
        if (s + NS - 1 < npanel) issue(s + NS - 1, lds + ((s + NS - 1) % NS) * CF::LDS_STAGE);
        if (scaled) {
            const int kb = (s * CF::BK) / 128;
            if (s > 0 && kb != kb_cur) {
                // new K scale block: keep acc divided by the current scale product
#pragma unroll
                for (int i = 0; i < CF::TM; ++i)
#pragma unroll
                    for (int j = 0; j < CF::TN; ++j) {
                        const int r0 = m0 + wm0 + 32 * i, c0 = n0 + wn0 + 32 * j;
                        const float ratio = block_scale(a, r0, c0, kb_cur) / block_scale(a, r0, c0, kb);
#pragma unroll
                        for (int r = 0; r < 16; ++r) acc[i][j][r] *= ratio;
                    }
                kb_cur = kb;
            }
        }
        pk_mma<CF>(lds + (s % NS) * CF::LDS_STAGE, acc, wm0, wn0, lane);
    }

    const int h = lane >> 5, l32 = lane & 31;
    const bool full = (m0 + CF::BM <= a.M) && (n0 + CF::BN <= a.N);
    const bool read_c = (a.beta != 0.f);
#pragma unroll
    for (int i = 0; i < CF::TM; ++i)
#pragma unroll
        for (int j = 0; j < CF::TN; ++j) {
            const int r0 = m0 + wm0 + 32 * i, c0 = n0 + wn0 + 32 * j;
            const float sc = a.alpha * (scaled ? block_scale(a, r0, c0, kb_cur) : 1.f);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = r0 + 8 * (r >> 2) + 4 * h + (r & 3);
                const int col = c0 + l32;
                if (!full && (row >= a.M || col >= a.N)) continue;
                float* p = a.C + (int64_t)row * a.ldc + col;
                float v = sc * acc[i][j][r];
                if (read_c) v = fmaf(a.beta, *p, v);
                *p = v;
            }
        }
}

// ------------------------------------------------------------------ host side
namespace {

struct PSched {
    int dtype, mode, BM, BN, BK, WGM, WGN, lds, threads;
    void (*kernel)(PackedArgs);
};

#define TG_PSCHED(DT, MODE, BM, BN, BK, WGM, WGN, NS)                                             \
    {DT, MODE, BM, BN, BK, WGM, WGN, PCfg<MODE, BM, BN, BK, WGM, WGN, NS>::LDS_BYTES,              \
     PCfg<MODE, BM, BN, BK, WGM, WGN, NS>::NT, &packed_kernel<PCfg<MODE, BM, BN, BK, WGM, WGN, NS>>}

const PSched kPacked[] = {
    // two workgroups per CU (LDS <= 80 KB), 4 waves each
    TG_PSCHED(TGEMM_F32, MODE_F32, 128, 128, 32, 2, 2, 2),
    TG_PSCHED(TGEMM_F32, MODE_F32, 128, 128, 16, 2, 2, 4),
    TG_PSCHED(TGEMM_F32_BF16X3, MODE_X3, 256, 128, 16, 2, 2, 3),
    TG_PSCHED(TGEMM_BF16, MODE_BF16, 256, 128, 32, 2, 2, 3),
    TG_PSCHED(TGEMM_FP8_E4M3, MODE_FP8, 256, 128, 64, 2, 2, 3),
    // one workgroup per CU, 8 waves
    TG_PSCHED(TGEMM_F32, MODE_F32, 256, 256, 32, 2, 4, 2),
    TG_PSCHED(TGEMM_F32, MODE_F32, 256, 256, 16, 2, 4, 4),
    TG_PSCHED(TGEMM_F32, MODE_F32, 256, 128, 32, 2, 4, 3),
    TG_PSCHED(TGEMM_F32_BF16X3, MODE_X3, 256, 256, 32, 2, 4, 2),
    TG_PSCHED(TGEMM_F32_BF16X3, MODE_X3, 256, 128, 32, 2, 4, 3),
    TG_PSCHED(TGEMM_F32_BF16X3, MODE_X3, 128, 128, 32, 2, 2, 2),
    TG_PSCHED(TGEMM_BF16, MODE_BF16, 256, 256, 64, 2, 4, 2),
    TG_PSCHED(TGEMM_BF16, MODE_BF16, 256, 256, 32, 2, 4, 4),
    TG_PSCHED(TGEMM_BF16, MODE_BF16, 128, 128, 64, 2, 2, 2),
    TG_PSCHED(TGEMM_FP8_E4M3, MODE_FP8, 256, 256, 128, 2, 4, 2),
    TG_PSCHED(TGEMM_FP8_E4M3, MODE_FP8, 256, 256, 64, 2, 4, 4),
    TG_PSCHED(TGEMM_FP8_E4M3, MODE_FP8, 128, 128, 128, 2, 2, 2),
};
constexpr int kNumPacked = sizeof(kPacked) / sizeof(kPacked[0]);

// Registry entries (kernel pointer unused: packed schedules launch through
// run_packed); vec = 0 marks "packed, any alignment".
SchedDesc g_packed_desc[kNumPacked];
struct DescInit {
    DescInit()
    {
        for (int i = 0; i < kNumPacked; ++i) {
            const PSched& p = kPacked[i];
            g_packed_desc[i] = SchedDesc{p.dtype, p.BM, p.BN, p.BK, p.WGM, p.WGN, 0, p.lds, p.threads,
                                         nullptr};
        }
    }
} g_desc_init;

// Per (device, stream) packing workspace, grown on demand, freed at shutdown.
struct Workspace {
    void* ptr = nullptr;
    size_t bytes = 0;
};
std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, Workspace> g_ws;

}  // namespace

const SchedDesc* packed_schedules(int* n)
{
    *n = kNumPacked;
    return g_packed_desc;
}

// Bytes of packing workspace for a problem.
size_t packed_workspace_bytes(int64_t M, int64_t N, int64_t K, int dtype)
{
    const int64_t Mp = (M + kPackRows - 1) / kPackRows * kPackRows;
    const int64_t Np = (N + kPackRows - 1) / kPackRows * kPackRows;
    const int64_t Kp = (K + kPackK - 1) / kPackK * kPackK;
    const int64_t es = dtype == TGEMM_FP8_E4M3 ? 1 : dtype == TGEMM_F32 ? 4 : 2;
    const int64_t arrays = dtype == TGEMM_F32_BF16X3 ? 2 : 1;
    return (size_t)((Mp + Np) * Kp * es * arrays);
}

int packed_workspace(hipStream_t s, size_t bytes, void** out)
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_ws_mu);
    Workspace& w = g_ws[std::make_pair(dev, s)];
    if (w.bytes < bytes) {
        hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &st) == hipSuccess && st != hipStreamCaptureStatusNone)
            return TGEMM_CAPTURE_UNPLANNED;  // allocation is not allowed under capture
        if (w.ptr) (void)hipFree(w.ptr);
        w.ptr = nullptr;
        w.bytes = 0;
        if (hipMalloc(&w.ptr, bytes) != hipSuccess) return TGEMM_ALLOC_FAILED;
        w.bytes = bytes;
    }
    *out = w.ptr;
    return TGEMM_SUCCESS;
}

void packed_release(hipStream_t s)
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_ws_mu);
    auto it = g_ws.find(std::make_pair(dev, s));
    if (it == g_ws.end()) return;
    if (it->second.ptr) (void)hipFree(it->second.ptr);
    g_ws.erase(it);
}

void packed_shutdown()
{
    std::lock_guard<std::mutex> lk(g_ws_mu);
    for (auto& kv : g_ws)
        if (kv.second.ptr) (void)hipFree(kv.second.ptr);
    g_ws.clear();
}

// Pack A and B into `ws` and run packed schedule `pid` (index into kPacked).
int run_packed_ws(int pid, int64_t M, int64_t N, int64_t K, float alpha, const void* A, int64_t lda,
                  const float* sA, const void* B, int64_t ldb, const float* sB, float beta, float* C,
                  int64_t ldc, int group_m, int xcd_remap, void* ws, hipStream_t s)
{
    const PSched& p = kPacked[pid];
    const int64_t Mp = (M + kPackRows - 1) / kPackRows * kPackRows;
    const int64_t Np = (N + kPackRows - 1) / kPackRows * kPackRows;
    const int64_t Kp = (K + kPackK - 1) / kPackK * kPackK;
    const int64_t es = p.dtype == TGEMM_FP8_E4M3 ? 1 : p.dtype == TGEMM_F32 ? 4 : 2;
    char* base = static_cast<char*>(ws);
    char* Ap = base;
    char* Alo = p.mode == MODE_X3 ? Ap + Mp * Kp * es : nullptr;
    char* Bp = base + Mp * Kp * es * (p.mode == MODE_X3 ? 2 : 1);
    char* Blo = p.mode == MODE_X3 ? Bp + Np * Kp * es : nullptr;

    const int64_t groups_a = Mp * (Kp / 8);
    const unsigned ga = (unsigned)std::min<int64_t>((groups_a + 255) / 256, 65536);
    const dim3 gb((unsigned)(Np / 64), (unsigned)(Kp / 64));
    switch (p.mode) {
        case MODE_F32:
            hipLaunchKernelGGL(pack_rows_kernel<MODE_F32>, dim3(ga), dim3(256), 0, s, A, lda, (int)M,
                               (int)K, Ap, nullptr, (int)Mp, (int)Kp);
            hipLaunchKernelGGL(pack_cols_kernel<MODE_F32>, gb, dim3(256), 0, s, B, ldb, (int)K, (int)N,
                               Bp, nullptr, (int)Np, (int)Kp);
            break;
        case MODE_X3:
            hipLaunchKernelGGL(pack_rows_kernel<MODE_X3>, dim3(ga), dim3(256), 0, s, A, lda, (int)M,
                               (int)K, Ap, Alo, (int)Mp, (int)Kp);
            hipLaunchKernelGGL(pack_cols_kernel<MODE_X3>, gb, dim3(256), 0, s, B, ldb, (int)K, (int)N,
                               Bp, Blo, (int)Np, (int)Kp);
            break;
        case MODE_BF16:
            hipLaunchKernelGGL(pack_rows_kernel<MODE_BF16>, dim3(ga), dim3(256), 0, s, A, lda, (int)M,
                               (int)K, Ap, nullptr, (int)Mp, (int)Kp);
            hipLaunchKernelGGL(pack_cols_kernel<MODE_BF16>, gb, dim3(256), 0, s, B, ldb, (int)K,
                               (int)N, Bp, nullptr, (int)Np, (int)Kp);
            break;
        default:
            hipLaunchKernelGGL(pack_rows_kernel<MODE_FP8>, dim3(ga), dim3(256), 0, s, A, lda, (int)M,
                               (int)K, Ap, nullptr, (int)Mp, (int)Kp);
            hipLaunchKernelGGL(pack_cols_kernel<MODE_FP8>, gb, dim3(256), 0, s, B, ldb, (int)K, (int)N,
                               Bp, nullptr, (int)Np, (int)Kp);
            break;
    }
    PackedArgs a;
    a.A = Ap;
    a.Alo = Alo;
    a.B = Bp;
    a.Blo = Blo;
    a.C = C;
    a.sA = sA;
    a.sB = sB;
    a.ldc = ldc;
    a.lds_a = (K + 127) / 128;
    a.lds_b = (N + 127) / 128;
    a.M = (int)M;
    a.N = (int)N;
    a.K = (int)K;
    a.Kp = (int)Kp;
    a.alpha = alpha;
    a.beta = beta;
    a.tiles_m = (int)((M + p.BM - 1) / p.BM);
    a.tiles_n = (int)((N + p.BN - 1) / p.BN);
    a.group_m = group_m < 1 ? 1 : group_m;
    a.xcd_remap = xcd_remap ? 1 : 0;
    if ((int64_t)a.tiles_m * a.tiles_n > INT32_MAX) return TGEMM_NOT_SUPPORTED;
    hipLaunchKernelGGL(p.kernel, dim3((unsigned)(a.tiles_m * a.tiles_n)), dim3(p.threads), 0, s, a);
    return hipGetLastError() == hipSuccess ? TGEMM_SUCCESS : TGEMM_LAUNCH_FAILED;
}

int run_packed(int pid, int64_t M, int64_t N, int64_t K, float alpha, const void* A, int64_t lda,
               const float* sA, const void* B, int64_t ldb, const float* sB, float beta, float* C,
               int64_t ldc, int group_m, int xcd_remap, hipStream_t s)
{
    void* ws = nullptr;
    const int rc = packed_workspace(s, packed_workspace_bytes(M, N, K, kPacked[pid].dtype), &ws);
    if (rc != TGEMM_SUCCESS) return rc;
    return run_packed_ws(pid, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, group_m,
                         xcd_remap, ws, s);
}

}  // namespace tg
