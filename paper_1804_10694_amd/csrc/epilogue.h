// Fused epilogue of the gemm kernels: C = v + beta * C over the results one lane
// holds, where v is alpha times the accumulated sums (the update of the gemm
// statement, Tiramisu paper, Section I).
#pragma once
#include <stdint.h>
#include <hip/hip_runtime.h>

namespace tg {

// Writes the TM x TN blocks of AR results a lane holds.  val(i, j, v) puts the
// AR values of block (i, j) (alpha applied) into v.  Block (i, j) starts at
// row r0, column c0 of C as origin(i, j, r0, c0) sets them (the same in every
// lane of a wave); value r of a lane sits at row r0 + lane_row + rrow(r),
// column c0 + lane_col.
//
// The blocks go in chunks of up to CH values per lane (16 unless the caller
// has registers to spare).  With beta != 0 every
// read of C in a chunk is issued before the first one is used, so a chunk
// costs one memory round trip (a read under a branch of its own would cost one
// per element).  Each row of a block is a buffer range that ends at C's last
// element, and the lane's offset into it is the same for every row; a lane
// whose column lies at or past N gets an offset beyond every range, so
// elements outside M x N read as zero and are never written, without a branch.
// Offsets are 32-bit: with ldc >= 2^25 a plain per-element loop runs instead.
// beta == 0 never reads C.
template <int TM, int TN, int AR, int CH = 16, class Val, class Org, class RowOf>
__device__ __forceinline__ void write_c(float* C, int64_t ldc, int M, int N, float beta, int lane_row,
                                        int lane_col, const Val& val, const Org& origin, const RowOf& rrow)
{
    constexpr int NB = AR >= CH ? 1 : CH / AR;  // blocks per chunk
    constexpr int NBLK = TM * TN;
    if (ldc >= (int64_t(1) << 25)) {
#pragma unroll
        for (int b = 0; b < NBLK; ++b) {
            const int i = b / TN, j = b % TN;
            float v[AR];
            val(i, j, v);
            int r0, c0;
            origin(i, j, r0, c0);
#pragma unroll
            for (int r = 0; r < AR; ++r) {
                const int row = r0 + lane_row + rrow(r), col = c0 + lane_col;
                if (row >= M || col >= N) continue;
                float* p = C + (int64_t)row * ldc + col;
                float x = v[r];
                if (beta != 0.f) x = fmaf(beta, *p, x);
                *p = x;
            }
        }
        return;
    }
    const int ldc4 = (int)ldc * 4;
#pragma unroll
    for (int b0 = 0; b0 < NBLK; b0 += NB) {
        const float* base[NB];
        int64_t bytes[NB];
        int lo[NB];
        float v[NB][AR];
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            if (b0 + q >= NBLK) continue;
            const int i = (b0 + q) / TN, j = (b0 + q) % TN;
            int r0, c0;
            origin(i, j, r0, c0);
            r0 = __builtin_amdgcn_readfirstlane(r0);
            c0 = __builtin_amdgcn_readfirstlane(c0);
            // bytes from the block's first element to one past C's last one
            const int64_t left = (int64_t)(M - 1 - r0) * ldc + (N - c0);
            bytes[q] = r0 >= M || left <= 0 ? 0 : left * 4;
            base[q] = C + (int64_t)r0 * ldc + c0;
            lo[q] = (c0 + lane_col < N) ? lane_row * ldc4 + lane_col * 4 : (int)0x80000000u;
            val(i, j, v[q]);
        }
        // value r of block q: the range from its row (a uniform base and
        // length), at the lane's offset, which is the same for every r
        // (length capped below 2^31, above every in-range offset: ldc < 2^25)
        auto range = [&](int q, int r) {
            const int64_t len = bytes[q] - (int64_t)rrow(r) * ldc * 4;
            return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base[q]) + rrow(r) * ldc, 0,
                                                     len <= 0 ? 0 : (int)min(len, (int64_t)0x7fffffff), 0x00020000);
        };
        if (beta != 0.f) {
            float c[NB][AR];
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                if (b0 + q >= NBLK) continue;
#pragma unroll
                for (int r = 0; r < AR; ++r)
                    c[q][r] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(range(q, r), lo[q], 0, 0));
            }
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                if (b0 + q >= NBLK) continue;
#pragma unroll
                for (int r = 0; r < AR; ++r) v[q][r] = fmaf(beta, c[q][r], v[q][r]);
            }
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            if (b0 + q >= NBLK) continue;
#pragma unroll
            for (int r = 0; r < AR; ++r)
                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v[q][r]), range(q, r), lo[q], 0, 0);
        }
    }
}

}  // namespace tg
