// C ABI of the gemm library (declarations and contracts in include/tgemm.h).
//
// Host-side responsibilities: argument validation before any HIP call,
// degenerate cases, schedule selection (policy), tile-grid planning and the
// stream-ordered launch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

#include "../../include/tgemm.h"
#include "kargs.h"
#include "registry.h"
#include "select.h"

using namespace tg;

namespace tg {

std::mutex g_mu;

// ------------------------------------------------------------------ device
// One check per device id: the kernels are gfx950 code objects only.
static int g_dev_ok[64];  // 0 unknown, 1 ok, -1 unusable

int ensure_device(hipStream_t /*stream*/)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return TGEMM_NO_DEVICE;
    int st = __atomic_load_n(&g_dev_ok[dev], __ATOMIC_ACQUIRE);
    if (st == 0) {
        hipDeviceProp_t prop;
        st = -1;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess &&
            std::strncmp(prop.gcnArchName, "gfx950", 6) == 0)
            st = 1;
        __atomic_store_n(&g_dev_ok[dev], st, __ATOMIC_RELEASE);
    }
    return st == 1 ? TGEMM_SUCCESS : TGEMM_NO_DEVICE;
}

// -------------------------------------------------------------- validation
static bool dtype_known(int dtype) { return dtype >= TGEMM_F32 && dtype <= TGEMM_FP8_E4M3; }

int validate_gemm(int64_t M, int64_t N, int64_t K, float alpha, const void* A, int64_t lda,
                  const void* B, int64_t ldb, float beta, const float* C, int64_t ldc, int dtype)
{
    if (!dtype_known(dtype)) return TGEMM_NOT_SUPPORTED;
    if (M < 0 || N < 0 || K < 0) return TGEMM_INVALID_VALUE;
    if (M > INT32_MAX || N > INT32_MAX || K > INT32_MAX) return TGEMM_INVALID_VALUE;
    if (lda < (K > 1 ? K : 1) || ldb < (N > 1 ? N : 1) || ldc < (N > 1 ? N : 1))
        return TGEMM_INVALID_VALUE;
    if (M == 0 || N == 0) return TGEMM_SUCCESS;
    if (!C) return TGEMM_INVALID_VALUE;
    const bool reads_ab = (K > 0 && alpha != 0.f);
    if (reads_ab && (!A || !B)) return TGEMM_INVALID_VALUE;
    if (!std::isfinite(alpha) || !std::isfinite(beta)) return TGEMM_INVALID_VALUE;
    (void)beta;
    return TGEMM_SUCCESS;
}

static size_t elem_size(int dtype)
{
    switch (dtype) {
        case TGEMM_F32:
        case TGEMM_F32_BF16X3: return 4;
        case TGEMM_BF16: return 2;
        default: return 1;
    }
}

// Vectorised schedules load 16 bytes at a time along rows of A and B.
bool vec_ok(const void* A, int64_t lda, const void* B, int64_t ldb, int dtype)
{
    const size_t es = elem_size(dtype);
    const uintptr_t a = reinterpret_cast<uintptr_t>(A), b = reinterpret_cast<uintptr_t>(B);
    return (a % 16 == 0) && (b % 16 == 0) && ((lda * (int64_t)es) % 16 == 0) &&
           ((ldb * (int64_t)es) % 16 == 0);
}

int schedule_serves(int id, int dtype, bool vec_allowed)
{
    if (id < 0 || id >= num_schedules()) return TGEMM_NOT_SUPPORTED;
    const SchedDesc& d = schedule(id);
    if (d.dtype != dtype) return TGEMM_NOT_SUPPORTED;
    if (d.vec > 1 && !vec_allowed) return TGEMM_NOT_SUPPORTED;
    return TGEMM_SUCCESS;
}

GemmArgs make_args(const SchedDesc& d, int64_t M, int64_t N, int64_t K, float alpha,
                   const void* A, int64_t lda, const void* B, int64_t ldb, float beta, float* C,
                   int64_t ldc, int group_m, int xcd_remap)
{
    GemmArgs a;
    std::memset(&a, 0, sizeof(a));
    a.A = A;
    a.B = B;
    a.C = C;
    a.lda = lda;
    a.ldb = ldb;
    a.ldc = ldc;
    a.M = (int)M;
    a.N = (int)N;
    a.K = (int)K;
    a.alpha = alpha;
    a.beta = beta;
    a.tiles_m = (int)((M + d.BM - 1) / d.BM);
    a.tiles_n = (int)((N + d.BN - 1) / d.BN);
    a.group_m = group_m < 1 ? 1 : group_m;
    a.xcd_remap = xcd_remap ? 1 : 0;
    return a;
}

int run_scaled(int64_t M, int64_t N, int64_t K, float alpha, const void* A, int64_t lda,
               const float* sA, const void* B, int64_t ldb, const float* sB, float beta, float* C,
               int64_t ldc, int dtype, int id, int group_m, int xcd_remap, hipStream_t s)
{
    const int pid = packed_index(id);
    if (pid >= 0)
        return run_packed(pid, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, group_m,
                          xcd_remap, s);
    const SchedDesc& d = schedule(id);
    GemmArgs a = make_args(d, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, group_m, xcd_remap);
    a.sA = sA;
    a.sB = sB;
    a.lds_a = (K + 127) / 128;
    a.lds_b = (N + 127) / 128;
    (void)dtype;
    if ((int64_t)a.tiles_m * a.tiles_n > INT32_MAX) return TGEMM_NOT_SUPPORTED;
    return launch_gemm(d, a, s) == hipSuccess ? TGEMM_SUCCESS : TGEMM_LAUNCH_FAILED;
}

bool stream_capturing(hipStream_t s)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &st) == hipSuccess && st != hipStreamCaptureStatusNone;
}

int run_gemm(int id, int64_t M, int64_t N, int64_t K, float alpha, const void* A, int64_t lda,
             const void* B, int64_t ldb, float beta, float* C, int64_t ldc, int group_m,
             int xcd_remap, hipStream_t stream)
{
    const int pid = packed_index(id);
    if (pid >= 0)
        return run_packed(pid, M, N, K, alpha, A, lda, nullptr, B, ldb, nullptr, beta, C, ldc,
                          group_m, xcd_remap, stream);
    const SchedDesc& d = schedule(id);
    if (d.inplace && !inplace_reach_ok(d, lda, ldb)) return TGEMM_NOT_SUPPORTED;
    GemmArgs a = make_args(d, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, group_m, xcd_remap);
    if ((int64_t)a.tiles_m * a.tiles_n > INT32_MAX) return TGEMM_NOT_SUPPORTED;
    return launch_gemm(d, a, stream) == hipSuccess ? TGEMM_SUCCESS : TGEMM_LAUNCH_FAILED;
}

}  // namespace tg

// ------------------------------------------------------------------- C ABI
extern "C" {

const char* tgemm_status_string(int status)
{
    switch (status) {
        case TGEMM_SUCCESS: return "TGEMM_SUCCESS";
        case TGEMM_INVALID_VALUE: return "TGEMM_INVALID_VALUE";
        case TGEMM_NOT_SUPPORTED: return "TGEMM_NOT_SUPPORTED";
        case TGEMM_LAUNCH_FAILED: return "TGEMM_LAUNCH_FAILED";
        case TGEMM_ALLOC_FAILED: return "TGEMM_ALLOC_FAILED";
        case TGEMM_CAPTURE_UNPLANNED: return "TGEMM_CAPTURE_UNPLANNED";
        case TGEMM_INTERNAL: return "TGEMM_INTERNAL";
        case TGEMM_NO_DEVICE: return "TGEMM_NO_DEVICE";
        case TGEMM_SCRATCH_TOO_SMALL: return "TGEMM_SCRATCH_TOO_SMALL";
        default: return "TGEMM_UNKNOWN_STATUS";
    }
}

int tgemm(int64_t M, int64_t N, int64_t K, float alpha, const void* A, int64_t lda,
          const void* B, int64_t ldb, float beta, float* C, int64_t ldc, int dtype, void* stream)
{
    int rc = validate_gemm(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, dtype);
    if (rc != TGEMM_SUCCESS) return rc;
    if (M == 0 || N == 0) return TGEMM_SUCCESS;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((rc = ensure_device(s)) != TGEMM_SUCCESS) return rc;
    if (K == 0 || alpha == 0.f)
        return launch_scale_c((int)M, (int)N, beta, C, ldc, s) == hipSuccess ? TGEMM_SUCCESS
                                                                             : TGEMM_LAUNCH_FAILED;
    Choice ch;
    const bool capturing = stream_capturing(s);
    const bool vok = vec_ok(A, lda, B, ldb, dtype);
    rc = select_schedule(M, N, K, dtype, vok, &ch, !capturing);
    if (rc != TGEMM_SUCCESS) return rc;
    for (int attempt = 0; attempt < 2; ++attempt) {
        if (dtype == TGEMM_BF16 || dtype == TGEMM_FP8_E4M3)  // unscaled: every scale is 1
            rc = run_scaled(M, N, K, alpha, A, lda, nullptr, B, ldb, nullptr, beta, C, ldc, dtype,
                            ch.id, ch.group_m, ch.xcd_remap, s);
        else
            rc = run_gemm(ch.id, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ch.group_m,
                          ch.xcd_remap, s);
        // a packed schedule whose workspace would have to grow under capture, or an
        // in-place one whose rows lie past the reach of its buffer offsets: use the
        // rule's schedule without packing instead
        if (rc != TGEMM_CAPTURE_UNPLANNED && !(rc == TGEMM_NOT_SUPPORTED && schedule(ch.id).inplace)) return rc;
        if ((rc = direct_schedule(M, N, K, dtype, vok, &ch)) != TGEMM_SUCCESS) return rc;
    }
    return rc;
}

int tgemm_with_schedule(int64_t M, int64_t N, int64_t K, float alpha, const void* A, int64_t lda,
                        const void* B, int64_t ldb, float beta, float* C, int64_t ldc, int dtype,
                        int schedule_id, int group_m, int xcd_remap, void* stream)
{
    int rc = validate_gemm(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, dtype);
    if (rc != TGEMM_SUCCESS) return rc;
    if (group_m < 1 || group_m > 64) return TGEMM_INVALID_VALUE;
    if (M == 0 || N == 0) return TGEMM_SUCCESS;
    const bool reads_ab = (K > 0 && alpha != 0.f);
    rc = schedule_serves(schedule_id, dtype, !reads_ab || vec_ok(A, lda, B, ldb, dtype));
    if (rc != TGEMM_SUCCESS) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((rc = ensure_device(s)) != TGEMM_SUCCESS) return rc;
    if (!reads_ab)
        return launch_scale_c((int)M, (int)N, beta, C, ldc, s) == hipSuccess ? TGEMM_SUCCESS
                                                                             : TGEMM_LAUNCH_FAILED;
    if (dtype == TGEMM_BF16 || dtype == TGEMM_FP8_E4M3)
        return run_scaled(M, N, K, alpha, A, lda, nullptr, B, ldb, nullptr, beta, C, ldc, dtype,
                          schedule_id, group_m, xcd_remap, s);
    return run_gemm(schedule_id, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, group_m, xcd_remap, s);
}

int tgemm_scaled(int64_t M, int64_t N, int64_t K, float alpha, const void* A, int64_t lda,
                 const float* scaleA, const void* B, int64_t ldb, const float* scaleB, float beta,
                 float* C, int64_t ldc, int dtype, void* stream)
{
    if (dtype != TGEMM_BF16 && dtype != TGEMM_FP8_E4M3) return TGEMM_NOT_SUPPORTED;
    int rc = validate_gemm(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, dtype);
    if (rc != TGEMM_SUCCESS) return rc;
    if (M == 0 || N == 0) return TGEMM_SUCCESS;
    const bool reads_ab = (K > 0 && alpha != 0.f);
    if (reads_ab && (!scaleA || !scaleB)) return TGEMM_INVALID_VALUE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((rc = ensure_device(s)) != TGEMM_SUCCESS) return rc;
    if (!reads_ab)
        return launch_scale_c((int)M, (int)N, beta, C, ldc, s) == hipSuccess ? TGEMM_SUCCESS
                                                                             : TGEMM_LAUNCH_FAILED;
    Choice ch;
    const bool capturing = stream_capturing(s);
    const bool vok = vec_ok(A, lda, B, ldb, dtype);
    rc = select_schedule(M, N, K, dtype, vok, &ch, !capturing);
    if (rc != TGEMM_SUCCESS) return rc;
    rc = run_scaled(M, N, K, alpha, A, lda, scaleA, B, ldb, scaleB, beta, C, ldc, dtype, ch.id,
                    ch.group_m, ch.xcd_remap, s);
    if (rc != TGEMM_CAPTURE_UNPLANNED) return rc;
    if ((rc = direct_schedule(M, N, K, dtype, vok, &ch)) != TGEMM_SUCCESS) return rc;
    return run_scaled(M, N, K, alpha, A, lda, scaleA, B, ldb, scaleB, beta, C, ldc, dtype, ch.id,
                      ch.group_m, ch.xcd_remap, s);
}

int tgemm_quantize_tiles(int64_t rows, int64_t cols, const float* X, int64_t ldx, void* Q,
                         int64_t ldq, float* S, int dtype, void* stream)
{
    if (dtype != TGEMM_BF16 && dtype != TGEMM_FP8_E4M3) return TGEMM_NOT_SUPPORTED;
    if (rows < 0 || cols < 0 || rows > INT32_MAX || cols > INT32_MAX) return TGEMM_INVALID_VALUE;
    if (ldx < (cols > 1 ? cols : 1) || ldq < (cols > 1 ? cols : 1)) return TGEMM_INVALID_VALUE;
    if (rows == 0 || cols == 0) return TGEMM_SUCCESS;
    if (!X || !Q || !S) return TGEMM_INVALID_VALUE;
    const int64_t tiles = ((rows + 127) / 128) * ((cols + 127) / 128);
    if (tiles > INT32_MAX) return TGEMM_INVALID_VALUE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = ensure_device(s);
    if (rc != TGEMM_SUCCESS) return rc;
    return launch_quantize((int)rows, (int)cols, X, ldx, Q, ldq, S, dtype, s) == hipSuccess
               ? TGEMM_SUCCESS
               : TGEMM_LAUNCH_FAILED;
}

int tgemm_schedule_count(void) { return num_schedules(); }

int tgemm_schedule_info(int id, int* info)
{
    if (id < 0 || id >= num_schedules() || !info) return TGEMM_INVALID_VALUE;
    const SchedDesc& d = schedule(id);
    info[0] = d.dtype;
    info[1] = d.BM;
    info[2] = d.BN;
    info[3] = d.BK;
    info[4] = d.WGM;
    info[5] = d.WGN;
    info[6] = d.vec;
    info[7] = d.lds_bytes;
    info[8] = d.split;
    info[9] = d.mfma;
    info[10] = d.inplace;
    return TGEMM_SUCCESS;
}

int tgemm_tile_map(int64_t M, int64_t N, int BM, int BN, int group_m, int xcd_remap,
                   int32_t* tile_m, int32_t* tile_n, int32_t* full)
{
    if (M <= 0 || N <= 0 || BM <= 0 || BN <= 0 || group_m < 1) return TGEMM_INVALID_VALUE;
    if (!tile_m || !tile_n || !full) return TGEMM_INVALID_VALUE;
    const int64_t tm_count = (M + BM - 1) / BM, tn_count = (N + BN - 1) / BN;
    if (tm_count * tn_count > INT32_MAX) return TGEMM_INVALID_VALUE;
    const int T = (int)(tm_count * tn_count);
    for (int w = 0; w < T; ++w) {
        const TileCoord c = map_tile(w, (int)tm_count, (int)tn_count, group_m, xcd_remap);
        tile_m[w] = c.tm;
        tile_n[w] = c.tn;
        full[w] = ((int64_t)(c.tm + 1) * BM <= M && (int64_t)(c.tn + 1) * BN <= N) ? 1 : 0;
    }
    return TGEMM_SUCCESS;
}

}  // extern "C"
