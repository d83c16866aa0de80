// Measured matrix-core peak: a loop of independent MFMAs with nothing else in
// it, so that achieved throughput can be stated against what the chip
// delivers at its running clock as well as against the datasheet figure.
// Each wave keeps four accumulator chains; 2048 workgroups of four waves
// (eight waves per SIMD) leave the issue logic no gaps to fill.
#include <hip/hip_runtime.h>

#include "../../include/tgemm.h"

namespace tg {

int ensure_device(hipStream_t stream);

typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef int i32x8_t __attribute__((ext_vector_type(8)));

constexpr int kPeakBlocks = 2048, kPeakThreads = 256, kChains = 4;

template <int DT>
__global__ void __launch_bounds__(kPeakThreads, 2) mfma_loop_kernel(int64_t iters, float* sink)
{
    const int lane = threadIdx.x & 63;
    f32x16_t acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[c][r] = 0.f;
    const float x = 1e-3f * (float)(lane + 1);
    bf16x8_t hb;
    i32x8_t q;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        hb[e] = (__bf16)(x * (float)(e + 1));
        q[e] = 0x38383838 + lane;  // small e4m3 codes
    }
    for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            if constexpr (DT == TGEMM_F32) acc[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(x, x, acc[c], 0, 0, 0);
            else if constexpr (DT == TGEMM_BF16) acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hb, hb, acc[c], 0, 0, 0);
            else acc[c] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(q, q, acc[c], 0, 0, 0, 0, 0, 0);
        }
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < kChains; ++c)
#pragma unroll
        for (int r = 0; r < 16; ++r) s += acc[c][r];
    if (lane == 0) sink[blockIdx.x * (kPeakThreads / 64) + (threadIdx.x >> 6)] = s;
}

}  // namespace tg

extern "C" int tgemm_mfma_loop(int dtype, int64_t iters, float* sink, int64_t sink_len, double* flops,
                               void* stream)
{
    using namespace tg;
    if (dtype != TGEMM_F32 && dtype != TGEMM_BF16 && dtype != TGEMM_FP8_E4M3) return TGEMM_NOT_SUPPORTED;
    const int64_t waves = (int64_t)kPeakBlocks * (kPeakThreads / 64);
    if (iters < 0 || !sink || sink_len < waves) return TGEMM_INVALID_VALUE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = ensure_device(s);
    if (rc != TGEMM_SUCCESS) return rc;
    const double per = dtype == TGEMM_F32 ? 2.0 * 32 * 32 * 2 : dtype == TGEMM_BF16 ? 2.0 * 32 * 32 * 16
                                                                                     : 2.0 * 32 * 32 * 64;
    if (flops) *flops = per * (double)kChains * (double)iters * (double)waves;
    if (dtype == TGEMM_F32)
        hipLaunchKernelGGL(mfma_loop_kernel<TGEMM_F32>, dim3(kPeakBlocks), dim3(kPeakThreads), 0, s, iters, sink);
    else if (dtype == TGEMM_BF16)
        hipLaunchKernelGGL(mfma_loop_kernel<TGEMM_BF16>, dim3(kPeakBlocks), dim3(kPeakThreads), 0, s, iters, sink);
    else
        hipLaunchKernelGGL(mfma_loop_kernel<TGEMM_FP8_E4M3>, dim3(kPeakBlocks), dim3(kPeakThreads), 0, s, iters,
                           sink);
    return hipGetLastError() == hipSuccess ? TGEMM_SUCCESS : TGEMM_LAUNCH_FAILED;
}
