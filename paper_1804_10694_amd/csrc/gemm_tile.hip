// One-problem gemm kernels for gfx950 (F32 and split-bf16x3): one workgroup
// per macro-tile; the tile body lives in tile_f32x3.h.
#include <hip/hip_runtime.h>

#include "kargs.h"
#include "registry.h"
#include "tile_f32x3.h"
#include "../../include/tgemm.h"

namespace tg {

template <class CF>
__global__ void __launch_bounds__(CF::NT) gemm_kernel(GemmArgs a)
{
    __shared__ __attribute__((aligned(16))) char lds[CF::LDS_BYTES];
    const TileCoord tc = map_tile(blockIdx.x, a.tiles_m, a.tiles_n, a.group_m, a.xcd_remap);
    const int m0 = tc.tm * CF::BM, n0 = tc.tn * CF::BN;
    const bool full = (m0 + CF::BM <= a.M) && (n0 + CF::BN <= a.N);
    if (full) tile_body<CF, false>(a, m0, n0, lds);
    else tile_body<CF, true>(a, m0, n0, lds);
}

// C = beta*C (beta == 0 writes zeros without reading C).  Used for K == 0
// and alpha == 0, where A and B are not read.
__global__ void scale_c_kernel(int M, int N, float beta, float* C, int64_t ldc)
{
    const int64_t total = (int64_t)M * N;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx / N, j = idx % N;
        float* p = C + i * ldc + j;
        *p = (beta != 0.f) ? beta * *p : 0.f;
    }
}

hipError_t launch_scale_c(int M, int N, float beta, float* C, int64_t ldc, hipStream_t s)
{
    const int64_t total = (int64_t)M * N;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(scale_c_kernel, dim3((unsigned)blocks), dim3(256), 0, s, M, N, beta, C, ldc);
    return hipGetLastError();
}

hipError_t launch_gemm(const SchedDesc& d, const GemmArgs& a, hipStream_t s)
{
    const unsigned grid = (unsigned)a.tiles_m * (unsigned)a.tiles_n;
    hipLaunchKernelGGL(d.kernel, dim3(grid), dim3(d.threads), 0, s, a);
    return hipGetLastError();
}

#define TG_SCHED(DT, MODE, BM, BN, BK, WGM, WGN, VEC)                                         \
    {DT, BM, BN, BK, WGM, WGN, VEC, Cfg<MODE, BM, BN, BK, WGM, WGN, VEC>::LDS_BYTES,          \
     Cfg<MODE, BM, BN, BK, WGM, WGN, VEC>::NT, &gemm_kernel<Cfg<MODE, BM, BN, BK, WGM, WGN, VEC>>}

#define TG_SCHED_V(DT, MODE, BM, BN, BK, WGM, WGN) \
    TG_SCHED(DT, MODE, BM, BN, BK, WGM, WGN, 4), TG_SCHED(DT, MODE, BM, BN, BK, WGM, WGN, 1)

static const SchedDesc kTileSchedules[] = {
    // plain float32 on v_mfma_f32_32x32x2_f32
    TG_SCHED_V(TGEMM_F32, MODE_F32, 128, 128, 16, 2, 2),
    TG_SCHED_V(TGEMM_F32, MODE_F32, 128, 128, 32, 2, 2),
    TG_SCHED_V(TGEMM_F32, MODE_F32, 256, 128, 16, 2, 2),
    TG_SCHED_V(TGEMM_F32, MODE_F32, 128, 256, 16, 2, 2),
    TG_SCHED_V(TGEMM_F32, MODE_F32, 64, 64, 16, 2, 2),
    TG_SCHED_V(TGEMM_F32, MODE_F32, 64, 128, 32, 2, 2),
    // split-bf16x3 on v_mfma_f32_32x32x16_bf16
    TG_SCHED_V(TGEMM_F32_BF16X3, MODE_X3, 128, 128, 32, 2, 2),
    TG_SCHED_V(TGEMM_F32_BF16X3, MODE_X3, 256, 128, 32, 2, 2),
    TG_SCHED_V(TGEMM_F32_BF16X3, MODE_X3, 128, 256, 32, 2, 2),
    TG_SCHED_V(TGEMM_F32_BF16X3, MODE_X3, 256, 256, 32, 2, 2),
    TG_SCHED_V(TGEMM_F32_BF16X3, MODE_X3, 64, 64, 32, 2, 2),
    TG_SCHED_V(TGEMM_F32_BF16X3, MODE_X3, 128, 128, 64, 2, 2),
};
const SchedDesc* tile_schedules(int* n)
{
    *n = (int)(sizeof(kTileSchedules) / sizeof(kTileSchedules[0]));
    return kTileSchedules;
}

}  // namespace tg
