// Kernel argument blocks and the tile placement shared by the host planner
// and the device kernels (both must agree bit for bit on which workgroup
// computes which tile).
#pragma once
#include <stdint.h>
#include <hip/hip_runtime.h>

namespace tg {

enum Mode : int { MODE_F32 = 0, MODE_X3 = 1, MODE_BF16 = 2, MODE_FP8 = 3 };

// Number of XCDs of an MI355X; the hardware hands consecutive workgroup ids
// to the XCDs round-robin.
constexpr int kNumXcd = 8;

struct GemmArgs {
    const void* A;
    const void* B;
    float* C;
    const float* sA;   // per-128x128-tile scales (scaled modes only)
    const float* sB;
    int64_t lda, ldb, ldc;
    int64_t lds_a, lds_b;  // row strides of the scale grids
    int M, N, K;
    float alpha, beta;
    int tiles_m, tiles_n;
    int group_m;
    int xcd_remap;
};

struct TileCoord {
    int tm, tn;
};

// Tiling map of the Tiramisu paper (the map of a tiling command, Section III-C,
// as the introduction of Section V writes it: i0 = floor(i/T), i1 = i % T
// in each dimension): workgroup `wg` owns macro-tile (tm, tn) and computes rows
// [tm*BM, tm*BM+BM) x columns [tn*BN, tn*BN+BN).  The order in which tiles are
// handed out is a bijection of [0, tiles_m*tiles_n) built from two steps:
//   1. XCD remap: the workgroups an XCD receives (wg % 8 == x) get one
//      contiguous run of the linear tile order, so tiles that share A rows and
//      B columns run on the same XCD and hit its L2;
//   2. grouped order: runs of group_m tile rows are swept column by column, so
//      concurrently running tiles share a few A and B panels.
__host__ __device__ inline TileCoord map_tile(int wg, int tiles_m, int tiles_n, int group_m,
                                              int xcd_remap)
{
    const int T = tiles_m * tiles_n;
    int s = wg;
    if (xcd_remap) {
        const int x = wg % kNumXcd;
        const int local = wg / kNumXcd;
        const int base = T / kNumXcd;
        const int rem = T % kNumXcd;
        s = x * base + (x < rem ? x : rem) + local;
    }
    const int per_group = group_m * tiles_n;
    const int g = s / per_group;
    const int first_m = g * group_m;
    const int left = tiles_m - first_m;
    const int gsize = left < group_m ? left : group_m;
    const int within = s - g * per_group;
    TileCoord c;
    c.tm = first_m + within % gsize;
    c.tn = within / gsize;
    return c;
}

}  // namespace tg
