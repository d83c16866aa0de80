// Back-to-back gemm with the intermediate kept on chip (project addition; the
// paper's VGG block fuses its two layers so that the intermediate stays close
// to the arithmetic, Section VI-A):
//
//   T = act(A B)                 A: M x K, B: K x N1 (N1 <= 256)
//   E = alpha * T D + beta * E   D: N1 x N2, E: M x N2
//
// One workgroup owns 64 rows of the output.  Phase 1 computes its 64 x N1
// block of T with the in-place pipeline of tile_inplace.h (K panels of A and B
// straight from memory into LDS), applies act in registers and stores T into
// LDS as N1/16 panels of 16 columns in the packed A layout; T never goes to
// memory.  Phase 2 walks E's columns in chunks of 128: each chunk streams
// 16-row panels of D into LDS while the MFMAs take their A operands from the
// resident T panels, then writes alpha * acc + beta * E.  Phase 1's pipeline
// stages live in the bytes T later takes, so a workgroup holds T plus two
// 8 KB D stages: two workgroups per CU for N1 up to 256, three up to 128.  Columns of T at or
// past N1 are stored as zero, so that nothing read past N1 (whatever B holds
// there) can reach E.  T is kept in FP32; the x3 form splits it, like every
// operand, into bf16 high and low parts when it reads it from LDS.
#include <hip/hip_runtime.h>

#include "../../include/tgemm.h"
#include "kargs.h"
#include "registry.h"
#include "tile_inplace.h"

namespace tg {

int ensure_device(hipStream_t stream);

struct G2Args {
    const char* A;
    const char* B;
    const char* D;
    float* E;
    int64_t lda, ldb, ldd, lde;
    int M, N1, N2, K;
    float alpha, beta;
    int relu;
};

template <int MODE, int N1P>
struct G2Cfg {
    static constexpr int BM = 64, BK = 16, NT = 256;
    using P1 = ICfg<MODE, 64, N1P, 16, 1, 4, 2>;  // phase 1: a 64 x N1P block of T, 4 waves side by side
    using P2 = ICfg<MODE, 64, 128, 16, 1, 4, 2>;  // phase 2: a 64 x 128 chunk of E
    static constexpr int CHUNK = P2::BN;
    static constexpr int TPANEL = 64 * 16 * 4;    // one 16-column panel of T (packed A layout, 4 units a row)
    static constexpr int T_BYTES = (N1P / 16) * TPANEL;
    static constexpr int LDS_BYTES = T_BYTES + 2 * P2::LDS_B;
    static constexpr int WG_PER_CU = (160 * 1024) / LDS_BYTES;
    static_assert(P1::LDS_BYTES <= T_BYTES, "phase-1 stages fit where T goes");
    static_assert(P1::UK == 4 && P2::UK == 4, "T panels use the layout of 16-deep A panels");
    static_assert(LDS_BYTES <= 160 * 1024, "LDS");
};

template <class CF>
__device__ __forceinline__ void zero_acc(f32x16 (&acc)[CF::TM][CF::TN])
{
#pragma unroll
    for (int i = 0; i < CF::TM; ++i)
#pragma unroll
        for (int j = 0; j < CF::TN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
}

template <int MODE, int N1P>
constexpr int kG2Occ = G2Cfg<MODE, N1P>::WG_PER_CU;

template <int MODE, int N1P, bool VEC>
__global__ void __launch_bounds__(256, (kG2Occ<MODE, N1P>)) gemm2_kernel(G2Args g)
{
    using G = G2Cfg<MODE, N1P>;
    using P1 = typename G::P1;
    using P2 = typename G::P2;
    __shared__ __attribute__((aligned(1024))) char lds[G::LDS_BYTES];
    char* tbuf = lds;                    // resident T panels (phase 1: its stages)
    char* stages = lds;                  // phase-1 stages
    char* dstages = lds + G::T_BYTES;    // phase-2 stages

    const int t = threadIdx.x, lane = t & 63, h = lane >> 5, l32 = lane & 31;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int m0 = blockIdx.x * G::BM;

    // ---- phase 1: T block = act(A[m0:m0+64, :] B)
    {
        PackedArgs a{};
        a.A = g.A;
        a.lda = g.lda;
        a.B = g.B;
        a.ldb = g.ldb;
        a.M = g.M;
        a.N = g.N1;
        a.K = g.K;
        InplaceA<P1, VEC> al;
        al.init(a, m0, lane, wave, typename InplaceA<P1, VEC>::Geom());
        InplaceB<P1, VEC> bl;
        bl.init(a, 0, lane, wave);
        const int wn0 = wave * P1::WTN;
        f32x16 acc[P1::TM][P1::TN];
        zero_acc<P1>(acc);
        const int npanel = (g.K + G::BK - 1) / G::BK;
        al.issue(0, stages);
        bl.issue(0, stages + P1::LDS_A);
        for (int s = 0; s < npanel; ++s) {
            wait_vmcnt<0>();
            lds_barrier();
            if (s + 1 < npanel) {
                char* st = stages + ((s + 1) & 1) * P1::LDS_STAGE;
                al.issue(s + 1, st);
                bl.issue(s + 1, st + P1::LDS_A);
            }
            pk_mma<P1, InplaceOps<P1>>(stages + (s & 1) * P1::LDS_STAGE, acc, 0, wn0, lane);
        }
        // act(acc) -> T panels, over the phase-1 stages once every wave is done
        // with them; columns at or past N1 become zero
        wait_lds_reads();
        lds_barrier();
#pragma unroll
        for (int i = 0; i < P1::TM; ++i)
#pragma unroll
            for (int j = 0; j < P1::TN; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int row = 32 * i + 8 * (r >> 2) + 4 * h + (r & 3);
                    const int col = wn0 + 32 * j + l32;
                    float v = acc[i][j][r];
                    if (g.relu && v < 0.f) v = 0.f;  // max(v, 0); NaN stays NaN
                    if (col >= g.N1) v = 0.f;
                    *reinterpret_cast<float*>(tbuf + (col / 16) * G::TPANEL +
                                              pk_slot<4>(row, (col % 16) / 4) * 16 + (col % 4) * 4) = v;
                }
        __syncthreads();  // T complete and visible to every wave
    }

    // ---- phase 2: E[m0:m0+64, n0:n0+128] = alpha * T D[:, n0:n0+128] + beta * E
    PackedArgs d{};
    d.B = g.D;
    d.ldb = g.ldd;
    d.N = g.N2;
    d.K = g.N1;
    const int wn0 = wave * P2::WTN;
    const int npanel = (g.N1 + G::BK - 1) / G::BK;
    for (int n0 = 0; n0 < g.N2; n0 += G::CHUNK) {
        InplaceB<P2, VEC> dl;
        dl.init(d, n0, lane, wave);
        f32x16 acc[P2::TM][P2::TN];
        zero_acc<P2>(acc);
        dl.issue(0, dstages);
        for (int s = 0; s < npanel; ++s) {
            wait_vmcnt<0>();
            lds_barrier();
            if (s + 1 < npanel) dl.issue(s + 1, dstages + ((s + 1) & 1) * P2::LDS_B);
            const char* ta = tbuf + s * G::TPANEL;
            const char* lb = dstages + (s & 1) * P2::LDS_B;
            using OP = InplaceOps<P2>;
            typename OP::Ops ops[2];
            OP::load_a(ta, ops[0], 0, 0, lane);
            OP::load_b(lb, ops[0], 0, wn0, lane);
#pragma unroll
            for (int q = 0; q < P2::NG; ++q) {
                if (q + 1 < P2::NG) {
                    OP::load_a(ta, ops[(q + 1) & 1], q + 1, 0, lane);
                    OP::load_b(lb, ops[(q + 1) & 1], q + 1, wn0, lane);
                }
                OP::compute(ops[q & 1], acc);
            }
        }
        wait_lds_reads();
        lds_barrier();  // every wave is done with the stages before the next chunk refills them
        write_c<P2::TM, P2::TN, 16>(
            g.E, g.lde, g.M, g.N2, g.beta, 4 * h, l32,
            [&](int i, int j, float (&v)[16]) {
#pragma unroll
                for (int r = 0; r < 16; ++r) v[r] = g.alpha * acc[i][j][r];
            },
            [&](int i, int j, int& r0, int& c0) {
                r0 = m0 + 32 * i;
                c0 = n0 + wn0 + 32 * j;
            },
            [](int r) { return 8 * (r >> 2) + (r & 3); });
    }
}

namespace {

typedef void (*G2Kernel)(G2Args);

template <int MODE, int N1P>
G2Kernel pick(bool vec)
{
    return vec ? &gemm2_kernel<MODE, N1P, true> : &gemm2_kernel<MODE, N1P, false>;
}

}  // namespace
}  // namespace tg

extern "C" int tgemm_gemm2(int64_t M, int64_t N1, int64_t N2, int64_t K, float alpha, const float* A,
                           int64_t lda, const float* B, int64_t ldb, int act, const float* D, int64_t ldd,
                           float beta, float* E, int64_t lde, int dtype, void* stream)
{
    using namespace tg;
    if (M < 0 || N1 < 0 || N2 < 0 || K < 0) return TGEMM_INVALID_VALUE;
    if (act != TGEMM_ACT_NONE && act != TGEMM_ACT_RELU) return TGEMM_INVALID_VALUE;
    if (dtype != TGEMM_F32 && dtype != TGEMM_F32_BF16X3) return TGEMM_NOT_SUPPORTED;
    if (!(alpha == alpha) || !(beta == beta)) return TGEMM_INVALID_VALUE;
    if (lde < (N2 > 1 ? N2 : 1)) return TGEMM_INVALID_VALUE;
    if (N1 > 256) return TGEMM_NOT_SUPPORTED;
    if (M > INT32_MAX || N2 > INT32_MAX || K > INT32_MAX) return TGEMM_NOT_SUPPORTED;
    if (M == 0 || N2 == 0) return TGEMM_SUCCESS;
    if (!E) return TGEMM_INVALID_VALUE;
    const bool reads = K > 0 && N1 > 0 && alpha != 0.f;
    if (reads) {
        if (!A || !B || !D) return TGEMM_INVALID_VALUE;
        if (lda < K || ldb < N1 || ldd < N2) return TGEMM_INVALID_VALUE;
        // a 64-row block of A and a 16-row panel of B or D within a buffer's 32-bit offsets
        if (64 * lda * 4 > INT32_MAX || 16 * ldb * 4 > INT32_MAX || 16 * ldd * 4 > INT32_MAX)
            return TGEMM_NOT_SUPPORTED;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = ensure_device(s);
    if (rc != TGEMM_SUCCESS) return rc;
    if (!reads)  // T = act(0) = 0: E = beta * E
        return launch_scale_c((int)M, (int)N2, beta, E, lde, s) == hipSuccess ? TGEMM_SUCCESS
                                                                              : TGEMM_LAUNCH_FAILED;
    auto al16 = [](const void* p, int64_t ld) { return reinterpret_cast<uintptr_t>(p) % 16 == 0 && ld % 4 == 0; };
    const bool vec = al16(A, lda) && al16(B, ldb) && al16(D, ldd) && K % 4 == 0 && N1 % 4 == 0 && N2 % 4 == 0;
    G2Args g;
    g.A = reinterpret_cast<const char*>(A);
    g.B = reinterpret_cast<const char*>(B);
    g.D = reinterpret_cast<const char*>(D);
    g.E = E;
    g.lda = lda;
    g.ldb = ldb;
    g.ldd = ldd;
    g.lde = lde;
    g.M = (int)M;
    g.N1 = (int)N1;
    g.N2 = (int)N2;
    g.K = (int)K;
    g.alpha = alpha;
    g.beta = beta;
    g.relu = act == TGEMM_ACT_RELU ? 1 : 0;
    const bool x3 = dtype == TGEMM_F32_BF16X3;
    const bool wide = N1 > 128;
    G2Kernel k = x3 ? (wide ? pick<MODE_X3, 256>(vec) : pick<MODE_X3, 128>(vec))
                    : (wide ? pick<MODE_F32, 256>(vec) : pick<MODE_F32, 128>(vec));
    const int64_t blocks = (M + 63) / 64;
    hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(256), 0, s, g);
    return hipGetLastError() == hipSuccess ? TGEMM_SUCCESS : TGEMM_LAUNCH_FAILED;
}
