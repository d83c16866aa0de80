// In-place LDS pipeline tile (F32 and split-bf16x3): the NS-stage
// direct-to-LDS pipeline of tile_packed.h, with both operands read straight
// from the caller's row-major matrices instead of packed copies.
//
// Why: a problem with short K (a few hundred) spends its time waiting for
// panels, not multiplying.  The register-staged tile body of tile_f32x3.h has
// one panel in flight per workgroup; here NS - 1 panels are in flight without
// costing registers, and no packing pass is needed.  The price is that the
// operands sit in LDS as float32 in the caller's orientation: A as rows of K
// (K-contiguous, the packed A layout), B as rows of N (k-major).  The F32 MFMA
// takes them as they are; the x3 form splits each operand into its bf16 high
// and low parts when it reads it from LDS (array packing moved from the
// packing pass to the operand fetch, Section I).
//
// Loads come in two widths.  VEC: 16 bytes per lane (4 floats, one LDS unit),
// for A and B 16-byte aligned with lda, ldb, K and N multiples of 4 (so no
// unit straddles the end of a row).  Otherwise 4 bytes per lane: four times
// the load instructions, no alignment needed, and the masking below is exact
// per element.  Either way BM * lda * 4 and BK * ldb * 4 must stay below 2^31
// (the buffer offsets are 32-bit); the host checks all of this.
//
// Edges.  Each panel's loads go through a buffer resource that spans only the
// bytes the tile may read: rows of A below M (k < K of the last one), rows of
// B below K (columns below N of the last one).  Reads past that return zero;
// every offset is in the per-lane VGPR operand, since the hardware does not
// range-check the scalar offset.  Units (elements) of A at k >= K inside a
// valid row (the row's tail or the next row) are given an offset past the
// range in the last panel, so they read as zero too.  Columns of B at n >= N
// inside a valid row hold whatever follows in memory; they only reach
// accumulator columns that the epilogue never stores.
#pragma once
#include <hip/hip_runtime.h>

#include "tile_packed.h"

namespace tg {

template <int MODE_, int BM_, int BN_, int BK_, int WGM_, int WGN_, int NS_>
struct ICfg {
    static constexpr int MODE = MODE_, BM = BM_, BN = BN_, BK = BK_, WGM = WGM_, WGN = WGN_;
    static constexpr int NS = NS_;
    static constexpr int NT = 64 * WGM * WGN, NW = WGM * WGN;
    static constexpr int UK = BK / 4;                          // 16-byte units per A row per panel
    static constexpr int UN = BN / 4;                          // units per B row (one k)
    static constexpr int MK = (MODE == MODE_F32) ? 8 : 16;     // k per MFMA group
    static constexpr int HS = MK / 2;                          // k offset of lanes 32..63
    static constexpr int NG = BK / MK;
    static constexpr int WTM = BM / WGM, WTN = BN / WGN, TM = WTM / 32, TN = WTN / 32;
    static constexpr int MS = 32, AR = 16;                     // 32 x 32 MFMA blocks
    using Acc = f32x16;
    __device__ __forceinline__ static int out_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }
    __device__ __forceinline__ static int out_col(int lane) { return lane & 31; }
    static constexpr int NARR = 1;                             // float32 in LDS for both forms
    static constexpr int LDS_A = BM * BK * 4, LDS_B = BK * BN * 4;
    static constexpr int LDS_STAGE = LDS_A + LDS_B;
    static constexpr int LDS_BYTES = NS * LDS_STAGE;
    // 16-byte loads per wave per panel, and 4-byte ones
    static constexpr int A_INSTR = BM * UK / 64 / NW, B_INSTR = BK * UN / 64 / NW;
    static constexpr int A_INSTR4 = BM * BK / 64 / NW, B_INSTR4 = BK * BN / 64 / NW;
    static_assert(MODE == MODE_F32 || MODE == MODE_X3, "float32 operands");
    static_assert(NS >= 2, "two stages at least");
    static_assert(BK % MK == 0, "panels hold whole MFMA groups");
    static_assert(UK <= 16 && 16 % UK == 0, "A swizzle");
    static_assert(UN >= 16 && UN % 16 == 0, "B swizzle flips bit 3 of the unit inside a row");
    static_assert((BM * UK) % (64 * NW) == 0 && (BK * UN) % (64 * NW) == 0, "loads divide among waves");
    static_assert(BN % 64 == 0, "a 4-byte load instruction fills whole B rows");
    static_assert(WTM % 32 == 0 && WTN % 32 == 0, "whole blocks");
    static_assert(LDS_BYTES <= 160 * 1024, "LDS");
};

// 64 x 64 in-place tiles: 4 waves, 16-deep panels in two 8 KB stages, so that
// eight workgroups fit per CU: with K of a few hundred, workgroups in flight
// hide the panel latency better than deeper pipelines (measured on MI355X
// over 512 grouped problems in [16, 2048]^3:
// 16-deep panels in 2 stages, 8 workgroups per CU, beat 3 stages with 6, 4
// with 5 and 32-deep panels with 3 to 5 by 5-18%).
// f32 stops at 7 per CU and x3 at 6: the 16-byte loads on rows of any length
// (see InplaceA) and x3's operand split need more than the 64 registers a
// wave may hold at 8 (f32 with those loads at 7 per CU: 0.879 ms on the
// 512-problem set, against 0.905 for 16-byte loads on aligned rows only at 8).
template <int MODE>
using InplaceCfg64 = ICfg<MODE, 64, 64, 16, 2, 2, 2>;
template <int MODE>
constexpr int kInplaceCap = (MODE == MODE_F32) ? 7 : 6;
template <int MODE>
constexpr int kInplace64Occ = (160 * 1024) / InplaceCfg64<MODE>::LDS_BYTES > kInplaceCap<MODE>
                                  ? kInplaceCap<MODE>
                                  : (160 * 1024) / InplaceCfg64<MODE>::LDS_BYTES;
// 128 x 128 in-place tiles: 4 waves of 64 x 64, the same 16-deep panels in
// two 16 KB stages; three workgroups per CU in the grouped launch (for the
// registers of the 16-byte loads on rows of any length, and x3's operand
// split).  The one-problem kernels (gemm_inplace.hip) have no tile loop and
// need fewer registers: eight workgroups per CU on 64 x 64 tiles, four (f32)
// and three (x3) on 128 x 128.  Each panel byte feeds
// twice the MFMAs of a 64 x 64 tile, which halves the operand reads from L2
// and beyond.
template <int MODE>
using InplaceCfg128 = ICfg<MODE, 128, 128, 16, 2, 2, 2>;
template <int MODE>
constexpr int kInplace128Occ = 3;

// Direct-to-LDS buffer load of W bytes per lane (the width is an immediate of
// the instruction, hence the two spellings).
template <int W>
__device__ __forceinline__ void lds_load(__amdgpu_buffer_rsrc_t r, char* dst, int voff)
{
    auto* d = (__attribute__((address_space(3))) void*)dst;
    if constexpr (W == 16) __builtin_amdgcn_raw_ptr_buffer_load_lds(r, d, 16, voff, 0, 0, 0);
    else __builtin_amdgcn_raw_ptr_buffer_load_lds(r, d, 4, voff, 0, 0, 0);
}

// B unit u of LDS row k (k-major panel, UN units per row).  The MFMA operand
// reads take 32 consecutive columns of row k in lanes 0-31 and of row k + HS in
// lanes 32-63; flipping bit 3 of the unit on alternate HS-row blocks puts the
// two halves 128 bytes apart in the bank space.
template <class CF>
__device__ __forceinline__ int ip_bslot(int k, int u)
{
    return k * CF::UN + (u ^ (((k / CF::HS) & 1) * 8));
}

// A panels from the caller's A (row-major, K-contiguous) into the packed A
// layout (pk_slot rows of UK units).  A 16-byte load instruction fills 64
// units, a 4-byte one 16 units (lane l: element l % 4 of unit l / 4).
// ANY: the 16-byte form (VEC) serves rows of any length: the panels whose
// 16-byte units would run past the end of the matrix take 4-byte loads.
// Without it the 16-byte form needs K and N multiples of 4.  The grouped
// launch enables it; the back-to-back gemm, whose 16-byte form has aligned
// dimensions anyway, does not (the unused branch split its loop body and cost
// it 13%).
template <class CF, bool VEC, bool ANY = false>
struct InplaceA {
    struct Geom {};
    static constexpr bool kAnyRow = ANY;
    static constexpr int NI = VEC ? CF::A_INSTR : CF::A_INSTR4, UK = CF::UK;
    static constexpr int LOADS = NI;
    static constexpr int W = VEC ? 16 : 4;  // bytes per lane per load
    static constexpr int OOB = INT32_MIN;   // beyond any range here: reads zero

    const char* base;  // row m0 of A
    int row_bytes, rows, K, wave;
    int voff[NI];      // this lane's byte offset (row and k) for each load
    int ku[NI];        // first k this lane loads within a panel

    __device__ __forceinline__ void init(const PackedArgs& a, int m0, int lane, int wave_, const Geom&)
    {
        wave = wave_;
        row_bytes = (int)a.lda * 4;
        base = a.A + (int64_t)m0 * row_bytes;
        rows = a.M - m0 < CF::BM ? a.M - m0 : CF::BM;
        K = a.K;
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int ig = wave * NI + i;
            int row, k;
            if (VEC) {
                const int u = ((lane % UK) ^ (lane / 16) ^ (4 * ig)) & (UK - 1);
                row = ig * (64 / UK) + lane / UK;
                k = 4 * u;
            } else {
                const int slot = ig * 16 + lane / 4;  // physical unit: row * UK + column
                row = slot / UK;
                const int u = (slot % UK) ^ ((row / (16 / UK)) & (UK - 1));  // pk_slot inverted
                k = 4 * u + lane % 4;
            }
            ku[i] = k;
            voff[i] = row * row_bytes + k * 4;
        }
    }

    __device__ __forceinline__ void issue(int panel, char* stage) const
    {
        const int k0 = panel * CF::BK;
        const __amdgpu_buffer_rsrc_t r = make_rsrc(base + k0 * 4, (rows - 1) * row_bytes + (K - k0) * 4);
        const bool tail = k0 + CF::BK > K;  // uniform
        if constexpr (VEC && kAnyRow) {
            if (tail && (K & 3)) {
                // a 16-byte unit would run past the end of its row: exact 4-byte loads
                issue4(r, k0, stage);
                return;
            }
        }
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int ig = wave * NI + i;
            lds_load<W>(r, stage + ig * 64 * W, (tail && k0 + ku[i] >= K) ? OOB : voff[i]);
        }
    }

    // The panel at k0 with 4-byte loads into the same layout (the offsets of
    // the 4-byte form, computed here: the tail panel is a tile's last).
    __device__ __forceinline__ void issue4(__amdgpu_buffer_rsrc_t r, int k0, char* stage) const
    {
        const int lane = threadIdx.x & 63;
#pragma unroll
        for (int i = 0; i < CF::A_INSTR4; ++i) {
            const int ig = wave * CF::A_INSTR4 + i;
            const int slot = ig * 16 + lane / 4;
            const int row = slot / UK;
            const int u = (slot % UK) ^ ((row / (16 / UK)) & (UK - 1));
            const int k = 4 * u + lane % 4;
            lds_load<4>(r, stage + ig * 64 * 4, k0 + k >= K ? OOB : row * row_bytes + k * 4);
        }
    }
};

// B panels (BK rows of the caller's row-major B) into the k-major LDS layout.
// A 16-byte load instruction fills 64 units, a 4-byte one 64 floats.
template <class CF, bool VEC, bool ANY = false>
struct InplaceB {
    static constexpr bool kAnyRow = ANY;
    static constexpr int NI = VEC ? CF::B_INSTR : CF::B_INSTR4;
    static constexpr int LOADS = NI;
    static constexpr int W = VEC ? 16 : 4;

    const char* base;  // column n0 of B
    int row_bytes, cols, K, wave;
    int voff[NI];

    __device__ __forceinline__ void init(const PackedArgs& a, int n0, int lane, int wave_)
    {
        wave = wave_;
        row_bytes = (int)a.ldb * 4;
        base = a.B + (int64_t)n0 * 4;
        cols = a.N - n0 < CF::BN ? a.N - n0 : CF::BN;
        K = a.K;
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int s = (wave * NI + i) * 64 + lane;  // LDS unit (VEC) or float this lane fills
            if (VEC) {
                const int k = s / CF::UN, up = s % CF::UN;
                const int u = up ^ (((k / CF::HS) & 1) * 8);
                voff[i] = k * row_bytes + u * 16;
            } else {
                const int k = s / CF::BN, d = s % CF::BN;
                const int u = (d / 4) ^ (((k / CF::HS) & 1) * 8);
                voff[i] = k * row_bytes + (4 * u + d % 4) * 4;
            }
        }
    }

    __device__ __forceinline__ void issue(int panel, char* stage) const
    {
        const int k0 = panel * CF::BK;
        const int rows = K - k0 < CF::BK ? K - k0 : CF::BK;
        // With N % 4 != 0 the last 16-byte unit of a row of an edge tile runs
        // past column N: into the next row of B for every row but the last, so
        // a panel that does not hold B's last row reads its rows whole (the
        // extra columns only feed outputs beyond N, which are never written),
        // and the panel that does takes exact 4-byte loads.
        const bool ragged = VEC && kAnyRow && (cols & 3);  // uniform
        if (ragged && k0 + CF::BK >= K) {
            issue4(make_rsrc(base + (int64_t)k0 * row_bytes, (rows - 1) * row_bytes + cols * 4), stage);
            return;
        }
        const __amdgpu_buffer_rsrc_t r = make_rsrc(base + (int64_t)k0 * row_bytes,
                                                   ragged ? rows * row_bytes : (rows - 1) * row_bytes + cols * 4);
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int ig = wave * NI + i;
            lds_load<W>(r, stage + ig * 64 * W, voff[i]);
        }
    }

    // A panel with 4-byte loads into the same layout (offsets computed here).
    __device__ __forceinline__ void issue4(__amdgpu_buffer_rsrc_t r, char* stage) const
    {
        const int lane = threadIdx.x & 63;
#pragma unroll
        for (int i = 0; i < CF::B_INSTR4; ++i) {
            const int ig = wave * CF::B_INSTR4 + i;
            const int s = ig * 64 + lane;
            const int k = s / CF::BN, d = s % CF::BN;
            const int u = (d / 4) ^ (((k / CF::HS) & 1) * 8);
            lds_load<4>(r, stage + ig * 64 * 4, k * row_bytes + (4 * u + d % 4) * 4);
        }
    }
};

template <class CF, int MODE = CF::MODE>
struct InplaceOps;

// F32: lane half h takes k = 8g + 4h + e (e = 0..3) for MFMA e of group g: one
// 16-byte A unit per block, four B values per block.
template <class CF>
struct InplaceOps<CF, MODE_F32> {
    struct Ops {
        u32x4 a[CF::TM];
        float b[CF::TN][4];
    };
    static constexpr int NREAD = CF::TM + 4 * CF::TN;
    static constexpr int NMFMA = 4 * CF::TM * CF::TN;

    // A operands from an A panel `la` (packed layout), B operands from a B panel `lb`
    __device__ __forceinline__ static void load_a(const char* la, Ops& o, int g, int wm0, int lane)
    {
        const int h = lane >> 5, l32 = lane & 31;
#pragma unroll
        for (int i = 0; i < CF::TM; ++i)
            o.a[i] = *reinterpret_cast<const u32x4*>(la + pk_slot<CF::UK>(wm0 + 32 * i + l32, 2 * g + h) * 16);
    }
    __device__ __forceinline__ static void load_b(const char* lb, Ops& o, int g, int wn0, int lane)
    {
        const int h = lane >> 5, l32 = lane & 31;
#pragma unroll
        for (int j = 0; j < CF::TN; ++j) {
            const int n = wn0 + 32 * j + l32;
#pragma unroll
            for (int e = 0; e < 4; ++e)
                o.b[j][e] = *reinterpret_cast<const float*>(
                    lb + ip_bslot<CF>(8 * g + 4 * h + e, n / 4) * 16 + (n % 4) * 4);
        }
    }
    __device__ __forceinline__ static void load(const char* stage, Ops& o, int g, int wm0, int wn0, int lane)
    {
        load_a(stage, o, g, wm0, lane);
        load_b(stage + CF::LDS_A, o, g, wn0, lane);
    }

    __device__ __forceinline__ static void compute(const Ops& o, f32x16 (&acc)[CF::TM][CF::TN])
    {
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int i = 0; i < CF::TM; ++i)
#pragma unroll
                for (int j = 0; j < CF::TN; ++j) {
                    const uint32_t xa = o.a[i][e];  // copied out before the bit cast
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(__builtin_bit_cast(float, xa), o.b[j][e],
                                                                     acc[i][j], 0, 0, 0);
                }
    }
};

// x3: lane half h takes k = 16g + 8h + e (e = 0..7): two A units and eight B
// values per block, each split into bf16 high and low parts on the way in.
template <class CF>
struct InplaceOps<CF, MODE_X3> {
    struct Ops {
        bf16x8 ah[CF::TM], al[CF::TM], bh[CF::TN], bl[CF::TN];
    };
    static constexpr int NREAD = 2 * CF::TM + 8 * CF::TN;
    static constexpr int NMFMA = 3 * CF::TM * CF::TN;

    __device__ __forceinline__ static void split8(const float (&x)[8], bf16x8& hi, bf16x8& lo)
    {
        split_bf16x8(x, hi, lo);
    }

    __device__ __forceinline__ static void load_a(const char* la, Ops& o, int g, int wm0, int lane)
    {
        const int h = lane >> 5, l32 = lane & 31;
#pragma unroll
        for (int i = 0; i < CF::TM; ++i) {
            const int row = wm0 + 32 * i + l32, u0 = 4 * g + 2 * h;
            const f32x4 p = *reinterpret_cast<const f32x4*>(la + pk_slot<CF::UK>(row, u0) * 16);
            const f32x4 q = *reinterpret_cast<const f32x4*>(la + pk_slot<CF::UK>(row, u0 + 1) * 16);
            const float x[8] = {p[0], p[1], p[2], p[3], q[0], q[1], q[2], q[3]};
            split8(x, o.ah[i], o.al[i]);
        }
    }
    __device__ __forceinline__ static void load_b(const char* lb, Ops& o, int g, int wn0, int lane)
    {
        const int h = lane >> 5, l32 = lane & 31;
#pragma unroll
        for (int j = 0; j < CF::TN; ++j) {
            const int n = wn0 + 32 * j + l32;
            float x[8];
#pragma unroll
            for (int e = 0; e < 8; ++e)
                x[e] = *reinterpret_cast<const float*>(lb + ip_bslot<CF>(16 * g + 8 * h + e, n / 4) * 16 + (n % 4) * 4);
            split8(x, o.bh[j], o.bl[j]);
        }
    }
    __device__ __forceinline__ static void load(const char* stage, Ops& o, int g, int wm0, int wn0, int lane)
    {
        load_a(stage, o, g, wm0, lane);
        load_b(stage + CF::LDS_A, o, g, wn0, lane);
    }

    __device__ __forceinline__ static void compute(const Ops& o, f32x16 (&acc)[CF::TM][CF::TN])
    {
        // small terms first: lo*hi, hi*lo, then hi*hi
#pragma unroll
        for (int i = 0; i < CF::TM; ++i)
#pragma unroll
            for (int j = 0; j < CF::TN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.al[i], o.bh[j], acc[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < CF::TM; ++i)
#pragma unroll
            for (int j = 0; j < CF::TN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.ah[i], o.bl[j], acc[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < CF::TM; ++i)
#pragma unroll
            for (int j = 0; j < CF::TN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.ah[i], o.bh[j], acc[i][j], 0, 0, 0);
    }
};

// One BM x BN macro-tile of problem `a` (a.A, a.lda, a.B, a.ldb: the caller's
// matrices) with the in-place pipeline; VEC selects 16-byte loads (on rows of
// any length, see InplaceA).
template <class CF, bool VEC>
__device__ __forceinline__ void inplace_tile(const PackedArgs& a, int m0, int n0, char* lds)
{
    constexpr bool any = VEC;
    packed_tile<CF, InplaceA<CF, VEC, any>, InplaceB<CF, VEC, any>, InplaceOps<CF>>(a, m0, n0, lds);
}

}  // namespace tg
