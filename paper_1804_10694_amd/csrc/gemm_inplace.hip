// One-problem gemm on in-place tiles (F32 and split-bf16x3): one workgroup per
// macro-tile of the tiling map (Section III-C; tile order as in kargs.h), K
// panels loaded from the caller's A and B straight into LDS by direct-to-LDS
// buffer loads (tile_inplace.h), so no packing pass runs.  Tile edges need no
// separate code path: loads past M, N or K return zero from the buffer range
// and the epilogue drops stores outside C (the full/partial tile split of
// Section V-A is done by the hardware's range check).  The small tiles' low
// LDS and register footprint lets several workgroups share a CU, which hides
// the panel latency on problems too small to keep the large packed tiles busy.
#include <hip/hip_runtime.h>

#include "kargs.h"
#include "registry.h"
#include "tile_inplace.h"
#include "../../include/tgemm.h"

namespace tg {

template <class CF, int OCC>
__global__ void __launch_bounds__(CF::NT, OCC) inplace_gemm_kernel(GemmArgs g)
{
    __shared__ __attribute__((aligned(1024))) char lds[CF::LDS_BYTES];
    PackedArgs a;
    a.A = static_cast<const char*>(g.A);
    a.Alo = nullptr;
    a.B = static_cast<const char*>(g.B);
    a.Blo = nullptr;
    a.C = g.C;
    a.sA = nullptr;
    a.sB = nullptr;
    a.ldc = g.ldc;
    a.lds_a = 0;
    a.lds_b = 0;
    a.lda = g.lda;
    a.ldb = g.ldb;
    a.M = g.M;
    a.N = g.N;
    a.K = g.K;
    a.Kp = 0;
    a.alpha = g.alpha;
    a.beta = g.beta;
    a.tiles_m = g.tiles_m;
    a.tiles_n = g.tiles_n;
    a.group_m = g.group_m;
    a.xcd_remap = g.xcd_remap;
    const TileCoord tc = map_tile(blockIdx.x, g.tiles_m, g.tiles_n, g.group_m, g.xcd_remap);
    // 16-byte loads at any 4-byte aligned address (float32 data always is)
    const bool vec = ((reinterpret_cast<uintptr_t>(g.A) | reinterpret_cast<uintptr_t>(g.B)) & 3) == 0;
    if (vec) inplace_tile<CF, true>(a, tc.tm * CF::BM, tc.tn * CF::BN, lds);
    else inplace_tile<CF, false>(a, tc.tm * CF::BM, tc.tn * CF::BN, lds);
}

#define TG_ISCHED(DT, CF, OCC) \
    {DT, CF::BM, CF::BN, CF::BK, CF::WGM, CF::WGN, 1, CF::LDS_BYTES, CF::NT, &inplace_gemm_kernel<CF, OCC>, 0, 32, 1}

static const SchedDesc kInplaceSchedules[] = {
    TG_ISCHED(TGEMM_F32, InplaceCfg64<MODE_F32>, kInplace64Occ<MODE_F32>),
    TG_ISCHED(TGEMM_F32, InplaceCfg128<MODE_F32>, kInplace128Occ<MODE_F32>),
    TG_ISCHED(TGEMM_F32_BF16X3, InplaceCfg64<MODE_X3>, kInplace64Occ<MODE_X3>),
    TG_ISCHED(TGEMM_F32_BF16X3, InplaceCfg128<MODE_X3>, kInplace128Occ<MODE_X3>),
};

const SchedDesc* inplace_schedules(int* n)
{
    *n = (int)(sizeof(kInplaceSchedules) / sizeof(kInplaceSchedules[0]));
    return kInplaceSchedules;
}

// A tile's rows of A and a panel's rows of B must lie within the 2^31-byte
// reach of a buffer offset.
bool inplace_reach_ok(const SchedDesc& d, int64_t lda, int64_t ldb)
{
    return (int64_t)d.BM * lda * 4 <= INT32_MAX && (int64_t)d.BK * ldb * 4 <= INT32_MAX;
}

}  // namespace tg
