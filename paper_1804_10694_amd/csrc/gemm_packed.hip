// Packed-operand gemm, one problem per launch, for every MFMA form: f32,
// split-bf16x3, and bf16 and e4m3 with per-tile scales.  A packing pre-pass
// (pack_rows_kernel for A, pack_cols_kernel for B^T) fills a workspace owned
// by the library per (device, stream); the main kernel runs one macro-tile per
// workgroup with the pipeline of tile_packed.h.  Packed rows are padded to
// multiples of kPackRows and K to a multiple of kPackK (packed_kp), so every
// schedule of the table reads whole tiles and whole panels.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/tgemm.h"
#include "kargs.h"
#include "registry.h"
#include "select.h"
#include "tile_f32x3.h"
#include "tile_packed.h"

namespace tg {

// Host helpers of api.cpp (argument checks, device check, launches).
int validate_gemm(int64_t M, int64_t N, int64_t K, float alpha, const void* A, int64_t lda,
                  const void* B, int64_t ldb, float beta, const float* C, int64_t ldc, int dtype);
int ensure_device(hipStream_t stream);
bool vec_ok(const void* A, int64_t lda, const void* B, int64_t ldb, int dtype);
int run_gemm(int id, int64_t M, int64_t N, int64_t K, float alpha, const void* A, int64_t lda,
             const void* B, int64_t ldb, float beta, float* C, int64_t ldc, int group_m,
             int xcd_remap, hipStream_t stream);
int run_scaled(int64_t M, int64_t N, int64_t K, float alpha, const void* A, int64_t lda,
               const float* sA, const void* B, int64_t ldb, const float* sB, float beta, float* C,
               int64_t ldc, int dtype, int id, int group_m, int xcd_remap, hipStream_t s);

// ------------------------------------------------------------------ kernels
// Groups of 8 k are numbered row by row; fewer than 2^32 of them (checked on
// the host), so the row and column come from one 32-bit division.
template <int MODE>
__global__ void pack_rows_kernel(const void* X, int64_t ldx, int R, int K, void* P, void* Plo,
                                 int Rp, int Kp, int vec)
{
    const uint32_t per_row = (uint32_t)Kp / 8, groups = (uint32_t)Rp * per_row;
    for (uint32_t gi = blockIdx.x * blockDim.x + threadIdx.x; gi < groups; gi += gridDim.x * blockDim.x) {
        const uint32_t r = gi / per_row;
        pack_row_group<MODE>(X, ldx, R, K, P, Plo, Kp, (int)r, (int)(gi - r * per_row) * 8, vec != 0);
    }
}

template <int MODE>
__global__ void __launch_bounds__(256) pack_cols_kernel(const void* X, int64_t ldx, int K, int N,
                                                        void* P, void* Plo, int Np, int Kp, int vec)
{
    __shared__ float tile[64][65];
    pack_col_block<MODE>(X, ldx, K, N, P, Plo, Np, Kp, blockIdx.x * 64, blockIdx.y * 64, tile, vec != 0);
}

template <class CF>
__global__ void __launch_bounds__(CF::NT, CF::WAVES_PER_EU) packed_kernel(PackedArgs a)
{
    static_assert(kPackK % CF::BK == 0 && CF::BM <= kPackRows && CF::BN <= kPackRows &&
                      kPackRows % CF::BM == 0 && kPackRows % CF::BN == 0,
                  "tiles and panels divide the packing padding");
    __shared__ __attribute__((aligned(1024))) char lds[CF::LDS_BYTES];
    const TileCoord tc = map_tile(blockIdx.x, a.tiles_m, a.tiles_n, a.group_m, a.xcd_remap);
    packed_tile<CF>(a, tc.tm * CF::BM, tc.tn * CF::BN, lds);
}

// ------------------------------------------------------------------ host side
namespace {

struct PSched {
    int dtype, mode, BM, BN, BK, WGM, WGN, lds, threads;
    void (*kernel)(PackedArgs);
};

#define TG_PSCHED(DT, MODE, BM, BN, BK, WGM, WGN, NS)                                             \
    {DT, MODE, BM, BN, BK, WGM, WGN, PCfg<MODE, BM, BN, BK, WGM, WGN, NS>::LDS_BYTES,              \
     PCfg<MODE, BM, BN, BK, WGM, WGN, NS>::NT, &packed_kernel<PCfg<MODE, BM, BN, BK, WGM, WGN, NS>>}

const PSched kPacked[] = {
    // two workgroups per CU (LDS <= 80 KB), 4 waves each
    TG_PSCHED(TGEMM_F32, MODE_F32, 128, 128, 32, 2, 2, 2),
    TG_PSCHED(TGEMM_F32, MODE_F32, 128, 128, 16, 2, 2, 4),
    // four workgroups per CU (LDS 32 KB): one wave of 128 x 128 tiles covers
    // 1024 tiles, for problems whose tile count falls just past 512
    TG_PSCHED(TGEMM_F32, MODE_F32, 128, 128, 16, 2, 2, 2),
    TG_PSCHED(TGEMM_F32_BF16X3, MODE_X3, 128, 128, 16, 2, 2, 2),
    TG_PSCHED(TGEMM_BF16, MODE_BF16, 128, 128, 32, 2, 2, 2),
    TG_PSCHED(TGEMM_FP8_E4M3, MODE_FP8, 128, 128, 64, 2, 2, 2),
    TG_PSCHED(TGEMM_F32_BF16X3, MODE_X3, 256, 128, 16, 2, 2, 3),
    TG_PSCHED(TGEMM_BF16, MODE_BF16, 256, 128, 32, 2, 2, 3),
    TG_PSCHED(TGEMM_FP8_E4M3, MODE_FP8, 256, 128, 64, 2, 2, 3),
    // two workgroups per CU of 8 waves, each wave 32 x 128 of the tile
    TG_PSCHED(TGEMM_F32, MODE_F32, 128, 256, 16, 4, 2, 3),
    // one workgroup per CU, 8 waves
    TG_PSCHED(TGEMM_F32, MODE_F32, 256, 256, 32, 2, 4, 2),
    TG_PSCHED(TGEMM_F32, MODE_F32, 256, 256, 16, 2, 4, 4),
    TG_PSCHED(TGEMM_F32, MODE_F32, 256, 128, 32, 2, 4, 3),
    TG_PSCHED(TGEMM_F32_BF16X3, MODE_X3, 256, 256, 32, 2, 4, 2),
    TG_PSCHED(TGEMM_F32_BF16X3, MODE_X3, 256, 128, 32, 2, 4, 3),
    TG_PSCHED(TGEMM_F32_BF16X3, MODE_X3, 128, 128, 32, 2, 2, 2),
    TG_PSCHED(TGEMM_BF16, MODE_BF16, 256, 256, 64, 2, 4, 2),
    TG_PSCHED(TGEMM_BF16, MODE_BF16, 256, 256, 32, 2, 4, 4),
    TG_PSCHED(TGEMM_BF16, MODE_BF16, 128, 128, 64, 2, 2, 2),
    TG_PSCHED(TGEMM_FP8_E4M3, MODE_FP8, 256, 256, 128, 2, 4, 2),
    TG_PSCHED(TGEMM_FP8_E4M3, MODE_FP8, 256, 256, 128, 4, 2, 2),
    TG_PSCHED(TGEMM_FP8_E4M3, MODE_FP8, 256, 256, 64, 2, 4, 4),
    TG_PSCHED(TGEMM_FP8_E4M3, MODE_FP8, 128, 128, 128, 2, 2, 2),
};
constexpr int kNumPacked = sizeof(kPacked) / sizeof(kPacked[0]);

// Registry entries (kernel pointer unused: packed schedules launch through
// run_packed); vec = 0 marks "packed, any alignment".
SchedDesc g_packed_desc[kNumPacked];
struct DescInit {
    DescInit()
    {
        for (int i = 0; i < kNumPacked; ++i) {
            const PSched& p = kPacked[i];
            g_packed_desc[i] = SchedDesc{p.dtype, p.BM, p.BN, p.BK, p.WGM, p.WGN, 0, p.lds, p.threads,
                                         nullptr};
        }
    }
} g_desc_init;

// Per (device, stream) packing workspace, grown on demand.  A buffer that is
// outgrown is retired, not freed: a HIP graph captured over an earlier call
// still holds its address and writes into it on every replay.  Retired
// buffers are freed at shutdown (or when their stream's workspace is released).
struct Workspace {
    void* ptr = nullptr;
    size_t bytes = 0;
    std::vector<void*> retired;
};
std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, Workspace> g_ws;

void free_workspace(Workspace& w)
{
    if (w.ptr) (void)hipFree(w.ptr);
    for (void* p : w.retired) (void)hipFree(p);
    w.ptr = nullptr;
    w.bytes = 0;
    w.retired.clear();
}

}  // namespace

const SchedDesc* packed_schedules(int* n)
{
    *n = kNumPacked;
    return g_packed_desc;
}

// Bytes of packing workspace for a problem.
size_t packed_workspace_bytes(int64_t M, int64_t N, int64_t K, int dtype)
{
    const int64_t Mp = (M + kPackRows - 1) / kPackRows * kPackRows;
    const int64_t Np = (N + kPackRows - 1) / kPackRows * kPackRows;
    const int64_t es = dtype == TGEMM_FP8_E4M3 ? 1 : dtype == TGEMM_F32 ? 4 : 2;
    const int64_t Kp = packed_kp(K, es);
    const int64_t arrays = dtype == TGEMM_F32_BF16X3 ? 2 : 1;
    return (size_t)((Mp + Np) * Kp * es * arrays);
}

int packed_workspace(hipStream_t s, size_t bytes, void** out)
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_ws_mu);
    Workspace& w = g_ws[std::make_pair(dev, s)];
    if (w.bytes < bytes) {
        hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &st) == hipSuccess && st != hipStreamCaptureStatusNone)
            return TGEMM_CAPTURE_UNPLANNED;  // allocation is not allowed under capture
        void* p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) return TGEMM_ALLOC_FAILED;
        if (w.ptr) w.retired.push_back(w.ptr);
        w.ptr = p;
        w.bytes = bytes;
    }
    *out = w.ptr;
    return TGEMM_SUCCESS;
}

// Only for streams whose calls were never captured (the autotuner's own stream).
void packed_release(hipStream_t s)
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_ws_mu);
    auto it = g_ws.find(std::make_pair(dev, s));
    if (it == g_ws.end()) return;
    free_workspace(it->second);
    g_ws.erase(it);
}

void packed_shutdown()
{
    std::lock_guard<std::mutex> lk(g_ws_mu);
    for (auto& kv : g_ws) free_workspace(kv.second);
    g_ws.clear();
}

namespace {
template <int MODE>
void pack_rows_mode(const void* X, int64_t ldx, int R, int K, void* P, void* Plo, int Rp, int Kp, int vec,
                    unsigned grid, hipStream_t s)
{
    hipLaunchKernelGGL(pack_rows_kernel<MODE>, dim3(grid), dim3(256), 0, s, X, ldx, R, K, P, Plo, Rp, Kp, vec);
}
template <int MODE>
void pack_cols_mode(const void* X, int64_t ldx, int K, int N, void* P, void* Plo, int Np, int Kp, int vec,
                    hipStream_t s)
{
    hipLaunchKernelGGL(pack_cols_kernel<MODE>, dim3((unsigned)(Np / 64), (unsigned)(Kp / 64)), dim3(256), 0, s,
                       X, ldx, K, N, P, Plo, Np, Kp, vec);
}
int mode_elem_bytes(int mode) { return mode == MODE_FP8 ? 1 : mode == MODE_BF16 ? 2 : 4; }
}  // namespace

int launch_pack_rows(int mode, const void* X, int64_t ldx, int64_t R, int64_t K, void* P, void* Plo,
                     int64_t Rp, int64_t Kp, hipStream_t s)
{
    if (R > Rp || K > Kp || Kp % 8 != 0 || Rp > INT32_MAX || Kp > INT32_MAX) return TGEMM_INTERNAL;
    // groups of 8 k are numbered in 32 bits, including the grid-stride overshoot
    const int64_t groups = Rp * (Kp / 8);
    if (groups >= ((int64_t)1 << 32) - 65536 * 256) return TGEMM_NOT_SUPPORTED;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((groups + 255) / 256, 65536));
    const int vec = pack_rows_vec(X, ldx, mode_elem_bytes(mode));
    switch (mode) {
        case MODE_F32: pack_rows_mode<MODE_F32>(X, ldx, (int)R, (int)K, P, Plo, (int)Rp, (int)Kp, vec, grid, s); break;
        case MODE_X3: pack_rows_mode<MODE_X3>(X, ldx, (int)R, (int)K, P, Plo, (int)Rp, (int)Kp, vec, grid, s); break;
        case MODE_BF16: pack_rows_mode<MODE_BF16>(X, ldx, (int)R, (int)K, P, Plo, (int)Rp, (int)Kp, vec, grid, s); break;
        case MODE_FP8: pack_rows_mode<MODE_FP8>(X, ldx, (int)R, (int)K, P, Plo, (int)Rp, (int)Kp, vec, grid, s); break;
        default: return TGEMM_INTERNAL;
    }
    return hipGetLastError() == hipSuccess ? TGEMM_SUCCESS : TGEMM_LAUNCH_FAILED;
}

int launch_pack_cols(int mode, const void* X, int64_t ldx, int64_t K, int64_t N, void* P, void* Plo,
                     int64_t Np, int64_t Kp, hipStream_t s)
{
    if (N > Np || K > Kp || Np % 64 != 0 || Kp % 64 != 0 || Np > INT32_MAX || Kp > INT32_MAX)
        return TGEMM_INTERNAL;
    if (Np / 64 > 0x7FFFFFFF || Kp / 64 > 65535) return TGEMM_NOT_SUPPORTED;
    const int vec = pack_cols_vec(X, ldx, mode_elem_bytes(mode));
    switch (mode) {
        case MODE_F32: pack_cols_mode<MODE_F32>(X, ldx, (int)K, (int)N, P, Plo, (int)Np, (int)Kp, vec, s); break;
        case MODE_X3: pack_cols_mode<MODE_X3>(X, ldx, (int)K, (int)N, P, Plo, (int)Np, (int)Kp, vec, s); break;
        case MODE_BF16: pack_cols_mode<MODE_BF16>(X, ldx, (int)K, (int)N, P, Plo, (int)Np, (int)Kp, vec, s); break;
        case MODE_FP8: pack_cols_mode<MODE_FP8>(X, ldx, (int)K, (int)N, P, Plo, (int)Np, (int)Kp, vec, s); break;
        default: return TGEMM_INTERNAL;
    }
    return hipGetLastError() == hipSuccess ? TGEMM_SUCCESS : TGEMM_LAUNCH_FAILED;
}

// Pack A and B into `ws` and run packed schedule `pid` (index into kPacked).
bool packed_k_ok(int64_t K, int dtype)
{
    const int64_t es = dtype == TGEMM_FP8_E4M3 ? 1 : dtype == TGEMM_F32 ? 4 : 2;
    return kPackRows * packed_kp(K, es) * es <= INT32_MAX;
}

int run_packed_ws(int pid, int64_t M, int64_t N, int64_t K, float alpha, const void* A, int64_t lda,
                  const float* sA, const void* B, int64_t ldb, const float* sB, float beta, float* C,
                  int64_t ldc, int group_m, int xcd_remap, void* ws, hipStream_t s)
{
    const PSched& p = kPacked[pid];
    if (!packed_k_ok(K, p.dtype)) return TGEMM_NOT_SUPPORTED;
    const int64_t Mp = (M + kPackRows - 1) / kPackRows * kPackRows;
    const int64_t Np = (N + kPackRows - 1) / kPackRows * kPackRows;
    const int64_t es = p.dtype == TGEMM_FP8_E4M3 ? 1 : p.dtype == TGEMM_F32 ? 4 : 2;
    const int64_t Kp = packed_kp(K, es);
    char* base = static_cast<char*>(ws);
    char* Ap = base;
    char* Alo = p.mode == MODE_X3 ? Ap + Mp * Kp * es : nullptr;
    char* Bp = base + Mp * Kp * es * (p.mode == MODE_X3 ? 2 : 1);
    char* Blo = p.mode == MODE_X3 ? Bp + Np * Kp * es : nullptr;

    int rc = launch_pack_rows(p.mode, A, lda, M, K, Ap, Alo, Mp, Kp, s);
    if (rc == TGEMM_SUCCESS) rc = launch_pack_cols(p.mode, B, ldb, K, N, Bp, Blo, Np, Kp, s);
    if (rc != TGEMM_SUCCESS) return rc;
    PackedArgs a;
    a.A = Ap;
    a.Alo = Alo;
    a.B = Bp;
    a.Blo = Blo;
    a.C = C;
    a.sA = sA;
    a.sB = sB;
    a.ldc = ldc;
    a.lds_a = (K + 127) / 128;
    a.lds_b = (N + 127) / 128;
    a.M = (int)M;
    a.N = (int)N;
    a.K = (int)K;
    a.Kp = (int)Kp;
    a.alpha = alpha;
    a.beta = beta;
    a.tiles_m = (int)((M + p.BM - 1) / p.BM);
    a.tiles_n = (int)((N + p.BN - 1) / p.BN);
    a.group_m = group_m < 1 ? 1 : group_m;
    a.xcd_remap = xcd_remap ? 1 : 0;
    if ((int64_t)a.tiles_m * a.tiles_n > INT32_MAX) return TGEMM_NOT_SUPPORTED;
    hipLaunchKernelGGL(p.kernel, dim3((unsigned)(a.tiles_m * a.tiles_n)), dim3(p.threads), 0, s, a);
    return hipGetLastError() == hipSuccess ? TGEMM_SUCCESS : TGEMM_LAUNCH_FAILED;
}

// ------------------------------------------------- no-allocation entry point
// Packing workspace of tgemm_noalloc: one static array per device, part of the
// library's code object, so it exists from the moment the library is loaded on
// a device until the process ends.  Host code never passes `scratch` itself to
// a kernel (in host code the name is a stand-in, not a device address): the
// device address comes from hipGetSymbolAddress, once per device, on the first
// call made with that device current.
static __device__ __align__(256) char scratch[TGEMM_NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[64];  // device address of `scratch`, per device id

int scratch_address(void** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return TGEMM_NO_DEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return TGEMM_LAUNCH_FAILED;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return TGEMM_SUCCESS;
}
}  // namespace

int run_packed(int pid, int64_t M, int64_t N, int64_t K, float alpha, const void* A, int64_t lda,
               const float* sA, const void* B, int64_t ldb, const float* sB, float beta, float* C,
               int64_t ldc, int group_m, int xcd_remap, hipStream_t s)
{
    if (!packed_k_ok(K, kPacked[pid].dtype)) return TGEMM_NOT_SUPPORTED;
    void* ws = nullptr;
    const int rc = packed_workspace(s, packed_workspace_bytes(M, N, K, kPacked[pid].dtype), &ws);
    if (rc != TGEMM_SUCCESS) return rc;
    return run_packed_ws(pid, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, group_m,
                         xcd_remap, ws, s);
}

}  // namespace tg

// tgemm without any allocation (declared in include/tgemm.h).
extern "C" int tgemm_noalloc(int64_t M, int64_t N, int64_t K, float alpha, const void* A, int64_t lda,
                             const void* B, int64_t ldb, float beta, float* C, int64_t ldc, int dtype,
                             void* stream)
{
    using namespace tg;
    int rc = validate_gemm(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, dtype);
    if (rc != TGEMM_SUCCESS) return rc;
    if (M == 0 || N == 0) return TGEMM_SUCCESS;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((rc = ensure_device(s)) != TGEMM_SUCCESS) return rc;
    if (K == 0 || alpha == 0.f)
        return launch_scale_c((int)M, (int)N, beta, C, ldc, s) == hipSuccess ? TGEMM_SUCCESS
                                                                             : TGEMM_LAUNCH_FAILED;
    // the cost model is never run here (a new prediction runs, and may allocate for, the
    // network); its cached answers, the tuning database and the rule are
    Choice ch;
    const bool vok = vec_ok(A, lda, B, ldb, dtype);
    if ((rc = select_schedule(M, N, K, dtype, vok, &ch, false)) != TGEMM_SUCCESS) return rc;
    const bool scaled = (dtype == TGEMM_BF16 || dtype == TGEMM_FP8_E4M3);
    const int pid = packed_index(ch.id);
    if (pid < 0) {  // direct schedules use no workspace
        if (scaled)
            return run_scaled(M, N, K, alpha, A, lda, nullptr, B, ldb, nullptr, beta, C, ldc, dtype, ch.id,
                              ch.group_m, ch.xcd_remap, s);
        return run_gemm(ch.id, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ch.group_m, ch.xcd_remap, s);
    }
    if (!packed_k_ok(K, dtype)) return TGEMM_NOT_SUPPORTED;
    if (packed_workspace_bytes(M, N, K, dtype) > (size_t)TGEMM_NOALLOC_SCRATCH_BYTES)
        return TGEMM_SCRATCH_TOO_SMALL;
    void* ws = nullptr;
    if ((rc = scratch_address(&ws)) != TGEMM_SUCCESS) return rc;
    return run_packed_ws(pid, M, N, K, alpha, A, lda, nullptr, B, ldb, nullptr, beta, C, ldc, ch.group_m,
                         ch.xcd_remap, ws, s);
}
