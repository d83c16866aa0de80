// Autotuner: chooses the tile schedule of a gemm by measurement (Tiramisu
// paper, Section VI-A: tile size and unrolling factor found by autotuning on
// the machine that runs the code).
//
// For one problem (M, N, K, dtype) every compiled schedule that serves the
// dtype is tried with every tile-order variant (group_m, XCD remap):
//   1. correctness gate: small-integer inputs, where every partial sum is an
//      exact integer, so the schedule's result must equal, bit for bit, the
//      result of a plain one-thread-per-element integer kernel (on a leading
//      sub-problem with the same tile structure when the problem is large);
//   2. warm-up, then `reps` launches timed one by one with HIP events; the
//      median is recorded.
// Each measurement is appended as one JSON line to the database file; keys
// already present (same problem, schedule, variant and schedule-table hash)
// are skipped, so an interrupted run resumes where it stopped.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <set>
#include <string>
#include <vector>

#include "../../include/tgemm.h"
#include "kargs.h"
#include "registry.h"
#include "select.h"

namespace tg {

int ensure_device(hipStream_t stream);
int run_gemm(int id, int64_t M, int64_t N, int64_t K, float alpha, const void* A, int64_t lda,
             const void* B, int64_t ldb, float beta, float* C, int64_t ldc, int group_m,
             int xcd_remap, hipStream_t stream);
int run_scaled(int64_t M, int64_t N, int64_t K, float alpha, const void* A, int64_t lda,
               const float* sA, const void* B, int64_t ldb, const float* sB, float beta, float* C,
               int64_t ldc, int dtype, int id, int group_m, int xcd_remap, hipStream_t s);
// FNV-1a over the schedule table: database lines from another table are ignored.
uint64_t schedule_space_hash()
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](int v) {
        for (int b = 0; b < 4; ++b) {
            h ^= (uint64_t)((v >> (8 * b)) & 0xff);
            h *= 1099511628211ull;
        }
    };
    for (int i = 0; i < num_schedules(); ++i) {
        const SchedDesc& d = schedule(i);
        mix(d.dtype); mix(d.BM); mix(d.BN); mix(d.BK); mix(d.WGM); mix(d.WGN); mix(d.vec);
        mix(d.lds_bytes); mix(d.split); mix(d.mfma); mix(d.inplace);
    }
    return h;
}

namespace {

// Small integers in [-8, 8] from a hash of the element index.
__device__ __forceinline__ int small_int(uint64_t idx, uint32_t seed)
{
    uint64_t x = idx * 0x9E3779B97F4A7C15ull + seed;
    x ^= x >> 31;
    x *= 0xBF58476D1CE4E5B9ull;
    x ^= x >> 29;
    return (int)(x % 17u) - 8;
}

// E4M3FN codes of 0..8 (sign bit added separately).
__constant__ uint8_t kE4m3Int[9] = {0x00, 0x38, 0x40, 0x44, 0x48, 0x4A, 0x4C, 0x4E, 0x50};

__global__ void fill_int_kernel(void* dst, int8_t* ints, int64_t n, uint32_t seed, int dtype)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int v = small_int((uint64_t)i, seed);
        ints[i] = (int8_t)v;
        if (dtype == TGEMM_F32 || dtype == TGEMM_F32_BF16X3) {
            static_cast<float*>(dst)[i] = (float)v;
        } else if (dtype == TGEMM_BF16) {
            static_cast<uint16_t*>(dst)[i] = (uint16_t)(__float_as_uint((float)v) >> 16);
        } else {
            const int a = v < 0 ? -v : v;
            static_cast<uint8_t*>(dst)[i] = (uint8_t)(kE4m3Int[a] | (v < 0 ? 0x80 : 0));
        }
    }
}

__global__ void fill_float_kernel(float* p, int64_t n, float v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Plain integer reference: one thread per element of C (gM x gN, compact), exact
// int64 sum over A (row stride lda) and B (row stride ldb).
__global__ void int_gemm_kernel(int gM, int gN, int gK, const int8_t* A, int64_t lda,
                                const int8_t* B, int64_t ldb, float* C)
{
    const int64_t total = (int64_t)gM * gN;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx / gN, j = idx % gN;
        long long s = 0;
        for (int k = 0; k < gK; ++k) s += (long long)A[i * lda + k] * B[(int64_t)k * ldb + j];
        C[idx] = (float)s;
    }
}

// Per-block count of elements of X (gM x gN, row stride ldx) whose bits differ
// from the compact reference Y.
__global__ void __launch_bounds__(256) mismatch_kernel(const float* X, int64_t ldx, const float* Y,
                                                       int gM, int gN, int* counts)
{
    __shared__ int red[256];
    int c = 0;
    const int64_t n = (int64_t)gM * gN;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        c += (__float_as_uint(X[(i / gN) * ldx + i % gN]) != __float_as_uint(Y[i])) ? 1 : 0;
    red[threadIdx.x] = c;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) counts[blockIdx.x] = red[0];
}

size_t elem_bytes(int dtype) { return dtype == TGEMM_BF16 ? 2 : (dtype == TGEMM_FP8_E4M3 ? 1 : 4); }

unsigned grid_for(int64_t n)
{
    int64_t b = (n + 255) / 256;
    return (unsigned)std::min<int64_t>(std::max<int64_t>(b, 1), 4096);
}

struct DevBuf {
    void* p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
    bool alloc(size_t bytes) { return hipMalloc(&p, bytes < 16 ? 16 : bytes) == hipSuccess; }
};

std::string key_of(int dtype, int64_t M, int64_t N, int64_t K, int sid, int gm, int xcd, uint64_t hash)
{
    char buf[160];
    std::snprintf(buf, sizeof(buf), "%d/%lld/%lld/%lld/%d/%d/%d/%llx", dtype, (long long)M,
                  (long long)N, (long long)K, sid, gm, xcd, (unsigned long long)hash);
    return buf;
}

bool json_int(const char* line, const char* key, long long* out)
{
    char pat[48];
    std::snprintf(pat, sizeof(pat), "\"%s\":", key);
    const char* p = std::strstr(line, pat);
    if (!p) return false;
    p += std::strlen(pat);
    while (*p == ' ') ++p;
    char* end = nullptr;
    const long long v = std::strtoll(p, &end, 10);
    if (end == p) return false;
    *out = v;
    return true;
}

bool json_hex(const char* line, const char* key, unsigned long long* out)
{
    char pat[48];
    std::snprintf(pat, sizeof(pat), "\"%s\": \"", key);
    const char* p = std::strstr(line, pat);
    if (!p) return false;
    p += std::strlen(pat);
    char* end = nullptr;
    const unsigned long long v = std::strtoull(p, &end, 16);
    if (end == p) return false;
    *out = v;
    return true;
}

// Keys already measured, plus their best valid time per key set.
void read_done(const char* path, uint64_t hash, std::set<std::string>* done)
{
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char line[4096];
    while (std::fgets(line, sizeof(line), f)) {
        if (!std::strchr(line, '\n') && !std::feof(f)) {
            int c;
            while ((c = std::fgetc(f)) != EOF && c != '\n') {}
            continue;
        }
        long long dt, m, n, k, sid, gm, xcd;
        unsigned long long h;
        if (!json_int(line, "dtype", &dt) || !json_int(line, "M", &m) || !json_int(line, "N", &n) ||
            !json_int(line, "K", &k) || !json_int(line, "sched", &sid) ||
            !json_int(line, "group_m", &gm) || !json_int(line, "xcd", &xcd) ||
            !json_hex(line, "space", &h))
            continue;
        if (h != hash) continue;
        done->insert(key_of((int)dt, m, n, k, (int)sid, (int)gm, (int)xcd, hash));
    }
    std::fclose(f);
}

}  // namespace

// The correctness gate runs on a leading sub-problem whose sizes keep their
// residues modulo 256 (every macro-tile and K panel size divides 256), so the
// schedule meets the same full/partial tile structure at a bounded cost.
static int64_t gate_dim(int64_t d) { return d <= 1024 ? d : 768 + d % 256; }

// Tile-order variants (group_m, XCD remap) tried for every compiled schedule:
// row-major and grouped sweeps, with and without the XCD remap.  The cost
// model ranks the same set (costmodel.hip).
static const int kOrderVariants[][2] = {{1, 0}, {4, 0}, {8, 0}, {2, 1}, {4, 1}, {8, 1}, {16, 1}, {32, 1}};

int autotune(int64_t M, int64_t N, int64_t K, int dtype, int reps, const char* db_path)
{
    if (M <= 0 || N <= 0 || K <= 0 || M > INT32_MAX || N > INT32_MAX || K > (1 << 18))
        return -TGEMM_INVALID_VALUE;  // K bound keeps integer partial sums below 2^24
    if (dtype < TGEMM_F32 || dtype > TGEMM_FP8_E4M3) return -TGEMM_NOT_SUPPORTED;
    if (reps < 1 || reps > 1000 || !db_path) return -TGEMM_INVALID_VALUE;
    int rc = ensure_device(nullptr);
    if (rc != TGEMM_SUCCESS) return -rc;

    const uint64_t hash = schedule_space_hash();
    std::set<std::string> done;
    read_done(db_path, hash, &done);

    const size_t es = elem_bytes(dtype);
    DevBuf A, B, C, R, Ai, Bi, SA, SB, cnt;
    const int64_t nA = M * K, nB = K * N, nC = M * N;
    const int64_t nsa = ((M + 127) / 128) * ((K + 127) / 128), nsb = ((K + 127) / 128) * ((N + 127) / 128);
    const int64_t gM = gate_dim(M), gN = gate_dim(N), gK = gate_dim(K);
    const unsigned cgrid = grid_for(gM * gN);
    if (!A.alloc(nA * es) || !B.alloc(nB * es) || !C.alloc(nC * 4) || !R.alloc(gM * gN * 4) ||
        !Ai.alloc(nA) || !Bi.alloc(nB) || !SA.alloc(nsa * 4) || !SB.alloc(nsb * 4) ||
        !cnt.alloc(cgrid * sizeof(int)))
        return -TGEMM_ALLOC_FAILED;

    hipStream_t s;
    if (hipStreamCreate(&s) != hipSuccess) return -TGEMM_LAUNCH_FAILED;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);

    hipLaunchKernelGGL(fill_int_kernel, dim3(grid_for(nA)), dim3(256), 0, s, A.p, (int8_t*)Ai.p, nA,
                       0x1234u, dtype);
    hipLaunchKernelGGL(fill_int_kernel, dim3(grid_for(nB)), dim3(256), 0, s, B.p, (int8_t*)Bi.p, nB,
                       0x9876u, dtype);
    hipLaunchKernelGGL(fill_float_kernel, dim3(grid_for(nsa)), dim3(256), 0, s, (float*)SA.p, nsa, 1.f);
    hipLaunchKernelGGL(fill_float_kernel, dim3(grid_for(nsb)), dim3(256), 0, s, (float*)SB.p, nsb, 1.f);
    hipLaunchKernelGGL(int_gemm_kernel, dim3(grid_for(gM * gN)), dim3(256), 0, s, (int)gM, (int)gN,
                       (int)gK, (const int8_t*)Ai.p, K, (const int8_t*)Bi.p, N, (float*)R.p);
    if (hipStreamSynchronize(s) != hipSuccess) {
        (void)hipStreamDestroy(s);
        return -TGEMM_LAUNCH_FAILED;
    }

    // (m, n, k) = the full problem for timing, the gate sub-problem for checking;
    // the row strides stay those of the full buffers.
    auto launch = [&](int sid, int gm, int xcd, float* out, int64_t m, int64_t n, int64_t k) {
        if (dtype == TGEMM_BF16 || dtype == TGEMM_FP8_E4M3)
            return run_scaled(m, n, k, 1.f, A.p, K, (const float*)SA.p, B.p, N, (const float*)SB.p,
                              0.f, out, N, dtype, sid, gm, xcd, s);
        return run_gemm(sid, m, n, k, 1.f, A.p, K, B.p, N, 0.f, out, N, gm, xcd, s);
    };

    // A run killed mid-line leaves a torn last line: start on a fresh line.
    bool torn = false;
    if (FILE* rf = std::fopen(db_path, "rb")) {
        if (std::fseek(rf, -1, SEEK_END) == 0) torn = std::fgetc(rf) != '\n';
        std::fclose(rf);
    }
    FILE* db = std::fopen(db_path, "a");
    if (!db) {
        (void)hipStreamDestroy(s);
        return -TGEMM_INVALID_VALUE;
    }
    if (torn) std::fputc('\n', db);
    const bool aligned = ((K * (int64_t)es) % 16 == 0) && ((N * (int64_t)es) % 16 == 0);
    const double flops = 2.0 * (double)M * (double)N * (double)K;
    int best = -1;
    double best_ms = 1e30;
    Choice best_choice{-1, 1, 0};
    std::vector<float> times(reps);
    std::vector<int> hcnt(cgrid);

    for (int sid = 0; sid < num_schedules(); ++sid) {
        const SchedDesc& d = schedule(sid);
        if (d.dtype != dtype || (d.vec > 1 && !aligned)) continue;
        for (const auto& ov : kOrderVariants) {
            const int gm = ov[0], xcd = ov[1];
            if (done.count(key_of(dtype, M, N, K, sid, gm, xcd, hash))) continue;
            // 1. correctness gate
            hipLaunchKernelGGL(fill_float_kernel, dim3(grid_for(nC)), dim3(256), 0, s, (float*)C.p, nC,
                               __builtin_nanf(""));
            bool valid = launch(sid, gm, xcd, (float*)C.p, gM, gN, gK) == TGEMM_SUCCESS;
            if (valid) {
                hipLaunchKernelGGL(mismatch_kernel, dim3(cgrid), dim3(256), 0, s, (const float*)C.p, N,
                                   (const float*)R.p, (int)gM, (int)gN, (int*)cnt.p);
                valid = hipMemcpyAsync(hcnt.data(), cnt.p, cgrid * sizeof(int), hipMemcpyDeviceToHost,
                                       s) == hipSuccess &&
                        hipStreamSynchronize(s) == hipSuccess;
                long long bad = 0;
                for (int c : hcnt) bad += c;
                valid = valid && bad == 0;
            }
            // 2. timing
            double med = -1.0;
            if (valid) {
                for (int w = 0; w < 2; ++w) launch(sid, gm, xcd, (float*)C.p, M, N, K);
                for (int r = 0; r < reps; ++r) {
                    (void)hipEventRecord(e0, s);
                    launch(sid, gm, xcd, (float*)C.p, M, N, K);
                    (void)hipEventRecord(e1, s);
                    (void)hipEventSynchronize(e1);
                    float ms = 0.f;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    times[r] = ms;
                }
                std::vector<float> sorted(times);
                std::sort(sorted.begin(), sorted.end());
                med = sorted[reps / 2];
                if (med < best_ms) {
                    best_ms = med;
                    best = sid;
                    best_choice = Choice{sid, gm, xcd};
                }
            }
            std::fprintf(db,
                         "{\"arch\": \"gfx950\", \"space\": \"%llx\", \"dtype\": %d, \"M\": %lld, "
                         "\"N\": %lld, \"K\": %lld, \"sched\": %d, \"BM\": %d, \"BN\": %d, \"BK\": %d, "
                         "\"WGM\": %d, \"WGN\": %d, \"vec\": %d, \"group_m\": %d, \"xcd\": %d, "
                         "\"reps\": %d, \"ms\": %.6f, \"tflops\": %.3f, \"valid\": %s}\n",
                         (unsigned long long)hash, dtype, (long long)M, (long long)N, (long long)K,
                         sid, d.BM, d.BN, d.BK, d.WGM, d.WGN, d.vec, gm, xcd, reps, med,
                         med > 0 ? flops / (med * 1e-3) / 1e12 : 0.0, valid ? "true" : "false");
            std::fflush(db);
        }
    }
    std::fclose(db);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    packed_release(s);
    (void)hipStreamDestroy(s);
    if (best >= 0) register_tuned(dtype, M, N, K, schedule(best).vec, best_choice, best_ms);
    // entries measured by an earlier, interrupted run count too
    (void)tgemm_load_tuning_db(db_path);
    Choice c;
    if (lookup_tuned(dtype, M, N, K, aligned ? 4 : 1, &c)) return c.id;
    return best >= 0 ? best : -TGEMM_INTERNAL;
}

}  // namespace tg

extern "C" int tgemm_autotune(int64_t M, int64_t N, int64_t K, int dtype, int reps, const char* db_path)
{
    return tg::autotune(M, N, K, dtype, reps, db_path);
}
