// 3x3 convolution layer as an implicit gemm (the paper's Conv benchmark layer,
// Section VI-A, and the observation there that sgemm is the building block of
// convolutions).
//
// Y[n, y, x, co] = alpha * sum_{dy, dx, ci} Xpad[n, y + dy, x + dx, ci] * Wt[dy, dx, ci, co]
//                  + beta * Y[n, y, x, co]
// with X, Y in NHWC, Wt as 3 x 3 x Cin x Cout, stride 1 and zero padding 1.
// As a gemm: M = batch * H * W output pixels, N = Cout, K = 9 * Cin; B = Wt
// read as a K x Cout row-major matrix, C = Y as an M x Cout row-major matrix,
// and A the im2col matrix, which is never materialised: while packing a K
// panel into LDS, each 16-byte unit of A (KU consecutive k of one output
// pixel) is read straight from the input pixel its tap points at, or set to
// zero where the tap falls into the padding.  Cin is a multiple of KU, so a
// unit never straddles two taps and is one vector load of KU channels.
//
// Everything else (LDS layout, MFMA register tiles, prefetch, full/partial
// tiles, fused epilogue) is the gemm tile body of tile_f32x3.h.
#include <hip/hip_runtime.h>

#include <cstring>

#include "../../include/tgemm.h"
#include "kargs.h"
#include "registry.h"
#include "tile_f32x3.h"

namespace tg {

int ensure_device(hipStream_t stream);

// NHWC input geometry; taps are 3 x 3 with padding 1, stride 1.
struct ConvGeom {
    int H, W, C;
};

template <class CF>
struct ConvPanel : Panel<CF> {
    using Geom = ConvGeom;
    static constexpr int KU = CF::KU, UK = CF::UK, NT = CF::NT;

    // Output pixel of each A unit this thread loads (its row r is fixed across
    // panels): flat index n*H*W + y*W + x (-1 past the last pixel), and y, x.
    int pix[CF::A_PER_T], py[CF::A_PER_T], px[CF::A_PER_T];

    __device__ __forceinline__ void init(const GemmArgs& a, int m0, int t, const Geom& g)
    {
#pragma unroll
        for (int p = 0; p < CF::A_PER_T; ++p) {
            const int m = m0 + (t + p * NT) / UK;
            const bool in = m < a.M;
            const int row = m / g.W;
            pix[p] = in ? m : -1;
            px[p] = m - row * g.W;
            py[p] = row % g.H;
        }
    }

    template <bool PRED>
    __device__ __forceinline__ void load(const GemmArgs& a, int m0, int n0, int k0, int t, const Geom& g)
    {
        const float* X = static_cast<const float*>(a.A);
#pragma unroll
        for (int p = 0; p < CF::A_PER_T; ++p) {
            const int kb = k0 + ((t + p * NT) % UK) * KU;
            typename Panel<CF>::fu v;
#pragma unroll
            for (int e = 0; e < KU; ++e) v[e] = 0.f;
            if (pix[p] >= 0 && kb < a.K) {
                const int tap = kb / g.C, ci = kb - tap * g.C;
                const int dy = tap / 3 - 1, dx = tap - (tap / 3) * 3 - 1;
                const int iy = py[p] + dy, ix = px[p] + dx;
                if (iy >= 0 && iy < g.H && ix >= 0 && ix < g.W) {
                    const float* src = X + (int64_t)(pix[p] + dy * g.W + dx) * g.C + ci;
#pragma unroll
                    for (int c = 0; c < KU / 4; ++c) {
                        const f32x4 q = *reinterpret_cast<const f32x4*>(src + 4 * c);
#pragma unroll
                        for (int e = 0; e < 4; ++e) v[4 * c + e] = q[e];
                    }
                }
            }
            this->ra[p] = v;
        }
        this->template load_b<PRED>(a, n0, k0, t);
    }
};

template <class CF>
__global__ void __launch_bounds__(CF::NT) conv3x3_kernel(GemmArgs a, ConvGeom g)
{
    __shared__ __attribute__((aligned(16))) char lds[CF::LDS_BYTES];
    const TileCoord tc = map_tile(blockIdx.x, a.tiles_m, a.tiles_n, a.group_m, a.xcd_remap);
    const int m0 = tc.tm * CF::BM, n0 = tc.tn * CF::BN;
    if (m0 + CF::BM <= a.M && n0 + CF::BN <= a.N) tile_body<CF, false, ConvPanel<CF>>(a, m0, n0, lds, g);
    else tile_body<CF, true, ConvPanel<CF>>(a, m0, n0, lds, g);
}

namespace {

struct ConvSched {
    int dtype, BM, BN, vec, threads;
    void (*kernel)(GemmArgs, ConvGeom);
};

#define TG_CONV(DT, MODE, BM, BN, BK, VEC) \
    {DT, BM, BN, VEC, Cfg<MODE, BM, BN, BK, 2, 2, VEC>::NT, &conv3x3_kernel<Cfg<MODE, BM, BN, BK, 2, 2, VEC>>}

// 128 x 128 tiles for layers with enough output pixels, 64 x 64 otherwise;
// 16-byte filter loads when Cout and the filter's address allow them.
const ConvSched kConv[] = {
    TG_CONV(TGEMM_F32, MODE_F32, 128, 128, 32, 4),        TG_CONV(TGEMM_F32, MODE_F32, 128, 128, 32, 1),
    TG_CONV(TGEMM_F32, MODE_F32, 64, 64, 16, 4),          TG_CONV(TGEMM_F32, MODE_F32, 64, 64, 16, 1),
    TG_CONV(TGEMM_F32_BF16X3, MODE_X3, 128, 128, 32, 4),  TG_CONV(TGEMM_F32_BF16X3, MODE_X3, 128, 128, 32, 1),
    TG_CONV(TGEMM_F32_BF16X3, MODE_X3, 64, 64, 32, 4),    TG_CONV(TGEMM_F32_BF16X3, MODE_X3, 64, 64, 32, 1),
};

}  // namespace

}  // namespace tg

extern "C" int tgemm_conv3x3(int64_t batch, int64_t H, int64_t W, int64_t Cin, int64_t Cout, float alpha,
                             const float* X, const float* Wt, float beta, float* Y, int dtype, void* stream)
{
    using namespace tg;
    if (batch < 0 || H < 0 || W < 0 || Cin < 0 || Cout < 0) return TGEMM_INVALID_VALUE;
    if (dtype != TGEMM_F32 && dtype != TGEMM_F32_BF16X3) return TGEMM_NOT_SUPPORTED;
    // the kernels index pixels, k and columns with 32-bit integers
    if (batch > INT32_MAX || H > INT32_MAX || W > INT32_MAX || Cin > INT32_MAX / 9 || Cout > INT32_MAX)
        return TGEMM_NOT_SUPPORTED;
    const int64_t HW = H * W;
    if (HW > INT32_MAX || (HW > 0 && batch > INT32_MAX / HW)) return TGEMM_NOT_SUPPORTED;
    const int64_t M = batch * HW, K = 9 * Cin;
    if (M == 0 || Cout == 0) return TGEMM_SUCCESS;
    if (!Y) return TGEMM_INVALID_VALUE;
    const bool reads_xw = K > 0 && alpha != 0.f;
    if (reads_xw && (!X || !Wt)) return TGEMM_INVALID_VALUE;
    // a 16-byte unit of A is KU channels of one input pixel
    const int ku = dtype == TGEMM_F32 ? 4 : 8;
    if (reads_xw && (Cin % ku != 0 || reinterpret_cast<uintptr_t>(X) % 16 != 0)) return TGEMM_NOT_SUPPORTED;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = ensure_device(s);
    if (rc != TGEMM_SUCCESS) return rc;
    if (!reads_xw)
        return launch_scale_c((int)M, (int)Cout, beta, Y, Cout, s) == hipSuccess ? TGEMM_SUCCESS
                                                                                 : TGEMM_LAUNCH_FAILED;

    const bool vec = (Cout % 4 == 0) && reinterpret_cast<uintptr_t>(Wt) % 16 == 0;
    const int tile = ((M + 127) / 128) * ((Cout + 127) / 128) >= 192 ? 128 : 64;
    const ConvSched* pick = nullptr;
    for (const ConvSched& c : kConv)
        if (c.dtype == dtype && c.BM == tile && c.vec == (vec ? 4 : 1)) pick = &c;
    if (!pick) return TGEMM_INTERNAL;

    GemmArgs a;
    std::memset(&a, 0, sizeof(a));
    a.A = X;
    a.B = Wt;
    a.C = Y;
    a.lda = K;
    a.ldb = Cout;
    a.ldc = Cout;
    a.M = (int)M;
    a.N = (int)Cout;
    a.K = (int)K;
    a.alpha = alpha;
    a.beta = beta;
    a.tiles_m = (int)((M + pick->BM - 1) / pick->BM);
    a.tiles_n = (int)((Cout + pick->BN - 1) / pick->BN);
    a.group_m = 8;
    a.xcd_remap = 1;
    const ConvGeom g{(int)H, (int)W, (int)Cin};
    if ((int64_t)a.tiles_m * a.tiles_n > INT32_MAX) return TGEMM_NOT_SUPPORTED;
    hipLaunchKernelGGL(pick->kernel, dim3((unsigned)(a.tiles_m * a.tiles_n)), dim3(pick->threads), 0, s, a, g);
    return hipGetLastError() == hipSuccess ? TGEMM_SUCCESS : TGEMM_LAUNCH_FAILED;
}
