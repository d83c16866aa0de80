// Convolution layer as an implicit gemm (the paper's Conv benchmark layer,
// Section VI-A, and the observation there that sgemm is the building block of
// convolutions), for R x R filters (R odd).  The 3 x 3 case is written below;
// for R x R read R*R taps and padding R / 2.  Every kernel exists twice: with
// R = 3 fixed at compile time (the paper credits its Conv result to such
// filter-size specialisation) and with R taken at run time.
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
// Two kernels share this scheme.  The direct one runs the gemm tile body of
// tile_f32x3.h (register-staged loads, full/partial tiles, fused epilogue).
// The packed one runs the LDS pipeline of tile_packed.h: the filter is packed
// once into K-contiguous rows of B^T (array packing, Section I), and each A
// panel is brought into LDS by 16-byte buffer loads whose per-lane offsets
// point at the input pixels of the lane's unit; units in the padding get an
// offset past the end of the buffer, which reads as zero.  The x3 form first
// splits X into its high and low bf16 parts (same NHWC layout), so both
// operands of every product come from memory as bf16.
#include <hip/hip_runtime.h>

#include <cstring>

#include "../../include/tgemm.h"
#include "kargs.h"
#include "registry.h"
#include "tile_f32x3.h"
#include "tile_packed.h"

namespace tg {

int ensure_device(hipStream_t stream);

// NHWC input geometry and the filter size R (odd; padding R / 2, stride 1).
struct ConvGeom {
    int H, W, C, R;
};

// Tap t of an R x R filter (row-major over dy, dx) as an offset from the output
// pixel.  FR > 0 fixes R at compile time (divisions by a constant); FR == 0
// takes R from the geometry.
template <int FR>
__device__ __forceinline__ void tap_offset(int tap, const ConvGeom& g, int& dy, int& dx)
{
    const int R = FR > 0 ? FR : g.R;
    const int q = tap / R;
    dy = q - R / 2;
    dx = tap - q * R - R / 2;
}

template <class CF, int FR>
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
                int dy, dx;
                tap_offset<FR>(tap, g, dy, dx);
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

template <class CF, int FR>
__global__ void __launch_bounds__(CF::NT) conv_kernel(GemmArgs a, ConvGeom g)
{
    __shared__ __attribute__((aligned(16))) char lds[CF::LDS_BYTES];
    const TileCoord tc = map_tile(blockIdx.x, a.tiles_m, a.tiles_n, a.group_m, a.xcd_remap);
    const int m0 = tc.tm * CF::BM, n0 = tc.tn * CF::BN;
    if (m0 + CF::BM <= a.M && n0 + CF::BN <= a.N) tile_body<CF, false, ConvPanel<CF, FR>>(a, m0, n0, lds, g);
    else tile_body<CF, true, ConvPanel<CF, FR>>(a, m0, n0, lds, g);
}

// A panels of the packed kernel, read from the NHWC input (X, or its bf16 hi
// and lo parts for x3) instead of packed rows.  Each lane of load instruction
// i fills the LDS slot that the packed layout assigns to it: row
// ig * (64 / UK) + lane / UK of the tile (ig = wave * A_INSTR + i) and the
// unit u of that row given by the swizzle of tile_packed.h (pk_slot), i.e.
// channels [ci, ci + KU) of tap `tap` for k = panel * BK + u * KU.
template <class CF, int FR>
struct ConvRowsA {
    using Geom = ConvGeom;
    static constexpr int NI = CF::A_INSTR, UK = CF::UK, KU = CF::KU;
    static constexpr int LOADS = CF::NARR * NI;  // loads per wave per panel
    static constexpr int OOB = INT32_MIN;  // offset 2^31: beyond any resource here, reads zero

    __amdgpu_buffer_rsrc_t r, rl;
    int wave, K, H, W, C;
    ConvGeom g;
    int ku[NI];                   // first k of this lane's unit within a panel
    int pix[NI], py[NI], px[NI];  // output pixel of this lane's row (-1 past M), its y and x

    __device__ __forceinline__ void init(const PackedArgs& a, int m0, int lane, int wave_, const Geom& geom)
    {
        wave = wave_;
        g = geom;
        K = a.K;
        H = g.H;
        W = g.W;
        C = g.C;
        const int bytes = a.M * C * CF::ES;  // below 2^31 (checked on the host)
        r = make_rsrc(a.A, bytes);
        rl = CF::MODE == MODE_X3 ? make_rsrc(a.Alo, bytes) : r;
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int ig = wave * NI + i;
            ku[i] = (((lane % UK) ^ (4 * ig + lane / 16)) & (UK - 1)) * KU;
            const int m = m0 + ig * (64 / UK) + lane / UK;
            const int row = m / W;
            pix[i] = m < a.M ? m : -1;
            px[i] = m - row * W;
            py[i] = row % H;
        }
    }

    __device__ __forceinline__ void issue(int panel, char* stage) const
    {
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int ig = wave * NI + i;
            const int k = panel * CF::BK + ku[i];
            const int tap = k / C, ci = k - tap * C;
            int dy, dx;
            tap_offset<FR>(tap, g, dy, dx);
            const int iy = py[i] + dy, ix = px[i] + dx;
            const bool in = pix[i] >= 0 && k < K && iy >= 0 && iy < H && ix >= 0 && ix < W;
            const int voff = in ? ((pix[i] + dy * W + dx) * C + ci) * CF::ES : OOB;
            auto* dst = (__attribute__((address_space(3))) void*)(stage + ig * 64 * 16);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(r, dst, 16, voff, 0, 0, 0);
            if (CF::MODE == MODE_X3) {
                auto* dlo = (__attribute__((address_space(3))) void*)(stage + CF::LDS_A + ig * 64 * 16);
                __builtin_amdgcn_raw_ptr_buffer_load_lds(rl, dlo, 16, voff, 0, 0, 0);
            }
        }
    }
};

template <class CF, int FR>
__global__ void __launch_bounds__(CF::NT, CF::WAVES_PER_EU) conv_packed_kernel(PackedArgs a, ConvGeom g)
{
    static_assert(kPackK % CF::BK == 0 && kPackRows % CF::BN == 0, "panels and tiles divide the packing padding");
    __shared__ __attribute__((aligned(1024))) char lds[CF::LDS_BYTES];
    const TileCoord tc = map_tile(blockIdx.x, a.tiles_m, a.tiles_n, a.group_m, a.xcd_remap);
    packed_tile<CF, ConvRowsA<CF, FR>>(a, tc.tm * CF::BM, tc.tn * CF::BN, lds, g);
}

namespace {

// Every kernel exists twice: specialised for 3 x 3 filters (FR = 3) and for a
// filter size given at run time (FR = 0).
struct ConvPacked {
    int dtype, mode, BM, BN, BK, NS, threads;
    void (*kernel[2])(PackedArgs, ConvGeom);  // [0]: 3 x 3, [1]: any R
};

#define TG_CONVP(DT, MODE, BM, BN, BK, WGM, WGN, NS)                         \
    {DT, MODE, BM, BN, BK, NS, PCfg<MODE, BM, BN, BK, WGM, WGN, NS>::NT,    \
     {&conv_packed_kernel<PCfg<MODE, BM, BN, BK, WGM, WGN, NS>, 3>,         \
      &conv_packed_kernel<PCfg<MODE, BM, BN, BK, WGM, WGN, NS>, 0>}}

// Tile shapes of the packed kernel.  Default (measured over 3x3 layers of
// 64 to 512 channels and 14 x 14 to 112 x 112 pixels): f32 takes shape 0
// (four workgroups per CU) everywhere; x3 takes shape 1 (256 x 256, eight
// waves) when Cout >= 256 and the layer has at least one 256 x 256 tile per
// CU, shape 0 otherwise.
const ConvPacked kConvPacked[] = {
    TG_CONVP(TGEMM_F32, MODE_F32, 128, 128, 16, 2, 2, 2),
    TG_CONVP(TGEMM_F32, MODE_F32, 128, 128, 16, 2, 2, 4),
    TG_CONVP(TGEMM_F32, MODE_F32, 256, 256, 32, 2, 4, 2),
    TG_CONVP(TGEMM_F32, MODE_F32, 256, 128, 32, 2, 4, 3),
    TG_CONVP(TGEMM_F32_BF16X3, MODE_X3, 128, 128, 32, 2, 2, 2),
    TG_CONVP(TGEMM_F32_BF16X3, MODE_X3, 256, 256, 32, 2, 4, 2),
    TG_CONVP(TGEMM_F32_BF16X3, MODE_X3, 256, 128, 32, 2, 4, 3),
    TG_CONVP(TGEMM_F32_BF16X3, MODE_X3, 128, 128, 16, 2, 2, 2),
};

int conv_default_shape(int dtype, int64_t M, int64_t Cout)
{
    if (dtype != TGEMM_F32_BF16X3) return 0;
    return Cout >= 256 && ((M + 255) / 256) * ((Cout + 255) / 256) >= 256 ? 1 : 0;
}

const ConvPacked* conv_packed(int dtype, int i)
{
    for (const ConvPacked& c : kConvPacked)
        if (c.dtype == dtype && i-- == 0) return &c;
    return nullptr;
}

struct ConvSched {
    int dtype, BM, BN, vec, threads;
    void (*kernel[2])(GemmArgs, ConvGeom);  // [0]: 3 x 3, [1]: any R
};

#define TG_CONV(DT, MODE, BM, BN, BK, VEC)                                      \
    {DT, BM, BN, VEC, Cfg<MODE, BM, BN, BK, 2, 2, VEC>::NT,                    \
     {&conv_kernel<Cfg<MODE, BM, BN, BK, 2, 2, VEC>, 3>, &conv_kernel<Cfg<MODE, BM, BN, BK, 2, 2, VEC>, 0>}}

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

namespace tg {
namespace {

// Kernel variant: 0 = specialised for 3 x 3, 1 = filter size at run time.
int variant(const ConvGeom& g, bool runtime_r) { return (g.R == 3 && !runtime_r) ? 0 : 1; }

int conv_direct(int64_t M, int64_t Cout, int64_t K, float alpha, const float* X, const float* Wt, float beta,
                float* Y, int dtype, const ConvGeom& g, bool runtime_r, hipStream_t s)
{
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
    if ((int64_t)a.tiles_m * a.tiles_n > INT32_MAX) return TGEMM_NOT_SUPPORTED;
    hipLaunchKernelGGL(pick->kernel[variant(g, runtime_r)], dim3((unsigned)(a.tiles_m * a.tiles_n)),
                       dim3(pick->threads), 0, s, a, g);
    return hipGetLastError() == hipSuccess ? TGEMM_SUCCESS : TGEMM_LAUNCH_FAILED;
}

// Whether the packed kernel can address the problem: X (or each bf16 part)
// and a 256-row block of packed filter rows must span fewer than 2^31 bytes.
bool conv_packed_ok(int64_t M, int64_t Cin, int64_t K, int dtype)
{
    const int64_t es = dtype == TGEMM_F32 ? 4 : 2;
    return M * Cin * es <= INT32_MAX && packed_k_ok(K, dtype);
}

int conv_packed_run(const ConvPacked& p, int64_t M, int64_t Cin, int64_t Cout, int64_t K, float alpha,
                    const float* X, const float* Wt, float beta, float* Y, const ConvGeom& g, bool runtime_r,
                    hipStream_t s)
{
    const int64_t Np = (Cout + kPackRows - 1) / kPackRows * kPackRows;
    const int64_t Kp = (K + kPackK - 1) / kPackK * kPackK;
    const bool x3 = p.mode == MODE_X3;
    const int64_t es = x3 ? 2 : 4, arrays = x3 ? 2 : 1;
    const int64_t wbytes = Np * Kp * es * arrays, xbytes = x3 ? 2 * M * Cin * es : 0;
    void* ws = nullptr;
    int rc = packed_workspace(s, (size_t)(wbytes + xbytes), &ws);
    if (rc != TGEMM_SUCCESS) return rc;
    char* Bp = static_cast<char*>(ws);
    char* Blo = x3 ? Bp + Np * Kp * es : nullptr;
    char* Ah = x3 ? Bp + wbytes : nullptr;
    char* Al = x3 ? Ah + M * Cin * es : nullptr;
    rc = launch_pack_cols(p.mode, Wt, Cout, K, Cout, Bp, Blo, Np, Kp, s);
    if (rc == TGEMM_SUCCESS && x3) rc = launch_pack_rows(MODE_X3, X, Cin, M, Cin, Ah, Al, M, Cin, s);
    if (rc != TGEMM_SUCCESS) return rc;

    PackedArgs a;
    std::memset(&a, 0, sizeof(a));
    a.A = x3 ? Ah : reinterpret_cast<const char*>(X);
    a.Alo = Al;
    a.B = Bp;
    a.Blo = Blo;
    a.C = Y;
    a.ldc = Cout;
    a.M = (int)M;
    a.N = (int)Cout;
    a.K = (int)K;
    a.Kp = (int)Kp;
    a.alpha = alpha;
    a.beta = beta;
    a.tiles_m = (int)((M + p.BM - 1) / p.BM);
    a.tiles_n = (int)((Cout + p.BN - 1) / p.BN);
    a.group_m = 8;
    a.xcd_remap = 1;
    if ((int64_t)a.tiles_m * a.tiles_n > INT32_MAX) return TGEMM_NOT_SUPPORTED;
    hipLaunchKernelGGL(p.kernel[variant(g, runtime_r)], dim3((unsigned)(a.tiles_m * a.tiles_n)),
                       dim3(p.threads), 0, s, a, g);
    return hipGetLastError() == hipSuccess ? TGEMM_SUCCESS : TGEMM_LAUNCH_FAILED;
}

int conv_run(int64_t batch, int64_t H, int64_t W, int64_t Cin, int64_t Cout, int64_t R, float alpha,
             const float* X, const float* Wt, float beta, float* Y, int dtype, int path, void* stream)
{
    if (batch < 0 || H < 0 || W < 0 || Cin < 0 || Cout < 0) return TGEMM_INVALID_VALUE;
    if (R < 1 || R % 2 == 0 || R > 31) return TGEMM_INVALID_VALUE;
    if (dtype != TGEMM_F32 && dtype != TGEMM_F32_BF16X3) return TGEMM_NOT_SUPPORTED;
    const bool runtime_r = (path & TGEMM_CONV_RUNTIME_R) != 0;
    path &= ~TGEMM_CONV_RUNTIME_R;
    const ConvPacked* packed = nullptr;
    if (path >= TGEMM_CONV_PACKED) {
        packed = conv_packed(dtype, path - TGEMM_CONV_PACKED);
        if (!packed) return TGEMM_INVALID_VALUE;
    } else if (path != TGEMM_CONV_AUTO && path != TGEMM_CONV_DIRECT) {
        return TGEMM_INVALID_VALUE;
    }
    // the kernels index pixels, k and columns with 32-bit integers
    if (batch > INT32_MAX || H > INT32_MAX || W > INT32_MAX || Cin > INT32_MAX / (R * R) || Cout > INT32_MAX)
        return TGEMM_NOT_SUPPORTED;
    const int64_t HW = H * W;
    if (HW > INT32_MAX || (HW > 0 && batch > INT32_MAX / HW)) return TGEMM_NOT_SUPPORTED;
    const int64_t M = batch * HW, K = R * R * Cin;
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
    const ConvGeom g{(int)H, (int)W, (int)Cin, (int)R};
    const bool packed_ok = conv_packed_ok(M, Cin, K, dtype);
    if (packed && !packed_ok) return TGEMM_NOT_SUPPORTED;
    if (path == TGEMM_CONV_AUTO && packed_ok) packed = conv_packed(dtype, conv_default_shape(dtype, M, Cout));
    if (packed) {
        rc = conv_packed_run(*packed, M, Cin, Cout, K, alpha, X, Wt, beta, Y, g, runtime_r, s);
        // under capture with no workspace yet: the direct kernel needs none
        if (!(rc == TGEMM_CAPTURE_UNPLANNED && path == TGEMM_CONV_AUTO)) return rc;
    }
    return conv_direct(M, Cout, K, alpha, X, Wt, beta, Y, dtype, g, runtime_r, s);
}

}  // namespace
}  // namespace tg

extern "C" int tgemm_conv3x3(int64_t batch, int64_t H, int64_t W, int64_t Cin, int64_t Cout, float alpha,
                             const float* X, const float* Wt, float beta, float* Y, int dtype, void* stream)
{
    return tg::conv_run(batch, H, W, Cin, Cout, 3, alpha, X, Wt, beta, Y, dtype, TGEMM_CONV_AUTO, stream);
}

extern "C" int tgemm_conv3x3_path(int64_t batch, int64_t H, int64_t W, int64_t Cin, int64_t Cout, float alpha,
                                  const float* X, const float* Wt, float beta, float* Y, int dtype, int path,
                                  void* stream)
{
    return tg::conv_run(batch, H, W, Cin, Cout, 3, alpha, X, Wt, beta, Y, dtype, path, stream);
}

extern "C" int tgemm_conv2d(int64_t batch, int64_t H, int64_t W, int64_t Cin, int64_t Cout, int64_t R, float alpha,
                            const float* X, const float* Wt, float beta, float* Y, int dtype, int path,
                            void* stream)
{
    return tg::conv_run(batch, H, W, Cin, Cout, R, alpha, X, Wt, beta, Y, dtype, path, stream);
}

extern "C" int tgemm_conv3x3_packed_shape(int dtype, int i, int* bm, int* bn, int* bk, int* stages)
{
    const tg::ConvPacked* p = i >= 0 ? tg::conv_packed(dtype, i) : nullptr;
    if (!p) return TGEMM_INVALID_VALUE;
    if (bm) *bm = p->BM;
    if (bn) *bn = p->BN;
    if (bk) *bk = p->BK;
    if (stages) *stages = p->NS;
    return TGEMM_SUCCESS;
}
