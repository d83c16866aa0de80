// Compiled tile schedules: the compile-time part of a schedule (tile sizes,
// wave grid, global-load width, precision mode).  The run-time part (tile
// order: group_m and the XCD remap) is passed in GemmArgs.
#pragma once
#include "kargs.h"

namespace tg {

struct SchedDesc {
    int dtype;      // tgemm_dtype this schedule serves
    int BM, BN, BK; // macro-tile (level-1 tiling) and K panel
    int WGM, WGN;   // wave grid: the macro-tile is split into WGM x WGN wave tiles
    int vec;        // global load width in float32 elements (4 or 1); 0 = packed operands
                    // (any alignment: a pre-pass packs A and B into a workspace)
    int lds_bytes;  // LDS footprint (both stages)
    int threads;
    void (*kernel)(GemmArgs);
    int split = 0;  // 1: stream-K (packed schedules): the (tile, K panel) iterations are split
                    // evenly over one wave of resident workgroups
    int mfma = 32;  // MFMA block: 32 (32 x 32 outputs) or 16 (16 x 16)
    int inplace = 0;  // 1: K panels go from the caller's A and B straight into LDS
                      // (direct-to-LDS loads, any 4-byte alignment; vec = 1)
};

// All compiled schedules, ids 0..num_schedules()-1 (tables of every kernel
// translation unit, concatenated in a fixed order).
int num_schedules();
const SchedDesc& schedule(int id);

// Per-translation-unit tables.
const SchedDesc* tile_schedules(int* n);    // F32 and split-bf16x3
const SchedDesc* scaled_schedules(int* n);  // bf16 and fp8 with per-tile scales
const SchedDesc* packed_schedules(int* n);  // packed-operand f32, x3, bf16, fp8
const SchedDesc* inplace_schedules(int* n); // in-place f32 and x3 (gemm_inplace.hip)
// Whether an in-place schedule reaches every row it loads with 32-bit buffer
// offsets for these row strides.
bool inplace_reach_ok(const SchedDesc& d, int64_t lda, int64_t ldb);

// Packed schedules (gemm_packed.hip): index within packed_schedules().
int run_packed(int pid, int64_t M, int64_t N, int64_t K, float alpha, const void* A, int64_t lda,
               const float* sA, const void* B, int64_t ldb, const float* sB, float beta, float* C,
               int64_t ldc, int group_m, int xcd_remap, hipStream_t s);
size_t packed_workspace_bytes(int64_t M, int64_t N, int64_t K, int dtype);
// Whether the packed kernels can address a problem of depth K: a tile's packed
// rows (256 of them, Kp elements each) must span fewer than 2^31 bytes, the
// reach of a buffer resource's 32-bit offsets.
bool packed_k_ok(int64_t K, int dtype);
void packed_shutdown();
void contract_shutdown();  // frees the contraction workspaces (contract.hip)
void packed_release(hipStream_t s);  // frees the workspace of one stream
// Per (device, stream) packing workspace of at least `bytes`, grown on demand
// (never under stream capture: TGEMM_CAPTURE_UNPLANNED).
int packed_workspace(hipStream_t s, size_t bytes, void** out);
// Packing passes of one operand form (MODE_*).  pack rows: R x K rows of X
// (row stride ldx) into Rp x Kp K-contiguous rows of P (and the low bf16
// halves into Plo for MODE_X3), zero past R and K.  pack cols: the K x N
// matrix X (row stride ldx) transposed into Np x Kp rows, zero past N and K.
// Kp is a multiple of 8 (of 64 for pack cols), Np of 64.
int launch_pack_rows(int mode, const void* X, int64_t ldx, int64_t R, int64_t K, void* P, void* Plo,
                     int64_t Rp, int64_t Kp, hipStream_t s);
int launch_pack_cols(int mode, const void* X, int64_t ldx, int64_t K, int64_t N, void* P, void* Plo,
                     int64_t Np, int64_t Kp, hipStream_t s);
constexpr int kPackRows = 256;  // packed row counts of the gemm path are multiples of this
constexpr int kPackK = 128;     // packed K of the gemm path is a multiple of this (elements)
// Packed row length (elements) of the gemm path for K and an element size of
// es bytes: K rounded up to kPackK, plus 512 bytes when that row pitch is a
// multiple of 4 KB.  With such a pitch the panel loads of all workgroups at
// one K position fall on the same few memory channels; the pad spreads them
// (measured on MI355X: x3 at 8192^3 +3%, e4m3 at 16384^3 +2%, bf16 even;
// pads of 128 or 256 bytes were slower for some of them).
constexpr int64_t packed_kp(int64_t K, int64_t es)
{
    const int64_t kp = (K + kPackK - 1) / kPackK * kPackK;
    return (kp * es) % 4096 == 0 ? kp + 512 / es : kp;
}
// Position of a schedule id inside packed_schedules(), or -1.
int packed_index(int id);

// Stream-ordered launches (defined in the HIP translation units).
hipError_t launch_gemm(const SchedDesc& d, const GemmArgs& a, hipStream_t s);
hipError_t launch_scale_c(int M, int N, float beta, float* C, int64_t ldc, hipStream_t s);
hipError_t launch_quantize(int rows, int cols, const float* X, int64_t ldx, void* Q, int64_t ldq,
                           float* S, int dtype, hipStream_t s);

}  // namespace tg
