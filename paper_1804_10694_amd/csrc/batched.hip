// Grouped gemm: many independent problems C_p = alpha_p A_p B_p + beta_p C_p
// in one persistent launch (project addition; the Tiramisu paper's sgemm is
// the building block of convolutions, Section VI-A, whose layers are batches
// of uneven gemms).
//
// Plan (host, once per problem set): every problem gets a tile configuration
// (macro-tile size and global-load width): 128 x 128 macro-tiles when both M
// and N reach a threshold, 64 x 64 otherwise.  The threshold is a built-in
// default unless tgemm_batched_autotune has measured the problem set's
// dimensions, in which case the fastest threshold it timed is used.
// Problems are ordered by the work of
// one of their tiles, largest first, and their tile counts are prefix-summed
// into one tile index space; a descriptor table and the prefix sums are
// uploaded to device memory the plan owns.  Launch: grid = the number of
// workgroups the device holds at once; workgroup w takes tiles w, w + grid,
// ... of the index space (heavy tiles first, light ones fill the tail), finds
// each tile's problem by binary search over the prefix sums and runs the
// matching tile body of tile_f32x3.h.  A launch allocates and uploads nothing,
// so it can be captured in a HIP graph once the plan exists.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <vector>

#include "../../include/tgemm.h"
#include "kargs.h"
#include "registry.h"
#include "tile_f32x3.h"

namespace tg {

int ensure_device(hipStream_t stream);
int validate_gemm(int64_t M, int64_t N, int64_t K, float alpha, const void* A, int64_t lda,
                  const void* B, int64_t ldb, float beta, const float* C, int64_t ldc, int dtype);
bool vec_ok(const void* A, int64_t lda, const void* B, int64_t ldb, int dtype);

struct GroupDesc {
    const void* A;
    const void* B;
    float* C;
    int64_t lda, ldb, ldc;
    int M, N, K;
    float alpha, beta;
    int cfg;         // index into GroupCfgs
    int tiles_m, tiles_n;
    int scale_only;  // K == 0 or alpha == 0: C = beta*C; A and B are not read
};

// Tile configurations of the grouped kernel: {64x64, 128x128} x {16-byte
// loads, 4-byte loads}.  The kernel's registers and LDS are the maximum over
// the four bodies.
template <int MODE>
struct GroupCfgs {
    static constexpr int BK_SMALL = (MODE == MODE_F32) ? 16 : 32;
    using C0 = Cfg<MODE, 64, 64, BK_SMALL, 2, 2, 4>;
    using C1 = Cfg<MODE, 64, 64, BK_SMALL, 2, 2, 1>;
    using C2 = Cfg<MODE, 128, 128, 32, 2, 2, 4>;
    using C3 = Cfg<MODE, 128, 128, 32, 2, 2, 1>;
    static constexpr int LDS = C2::LDS_BYTES > C0::LDS_BYTES ? C2::LDS_BYTES : C0::LDS_BYTES;
};
constexpr int kGroupTile[4] = {64, 64, 128, 128};

template <class CF>
__device__ __forceinline__ void run_tile(const GemmArgs& a, int local, char* lds)
{
    const TileCoord tc = map_tile(local, a.tiles_m, a.tiles_n, 8, 0);
    const int m0 = tc.tm * CF::BM, n0 = tc.tn * CF::BN;
    if (m0 + CF::BM <= a.M && n0 + CF::BN <= a.N) tile_body<CF, false>(a, m0, n0, lds);
    else tile_body<CF, true>(a, m0, n0, lds);
}

template <int MODE>
__global__ void __launch_bounds__(256) grouped_kernel(const GroupDesc* __restrict__ desc,
                                                      const int* __restrict__ prefix, int count,
                                                      int total)
{
    using G = GroupCfgs<MODE>;
    __shared__ __attribute__((aligned(16))) char lds[G::LDS];
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        // owner: the last problem whose first tile is <= t
        int lo = 0, hi = count - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (prefix[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        const GroupDesc& g = desc[lo];
        const int local = t - prefix[lo];
        GemmArgs a;
        a.A = g.A;
        a.B = g.B;
        a.C = g.C;
        a.sA = nullptr;
        a.sB = nullptr;
        a.lda = g.lda;
        a.ldb = g.ldb;
        a.ldc = g.ldc;
        a.lds_a = 0;
        a.lds_b = 0;
        a.M = g.M;
        a.N = g.N;
        a.K = g.K;
        a.alpha = g.alpha;
        a.beta = g.beta;
        a.tiles_m = g.tiles_m;
        a.tiles_n = g.tiles_n;
        a.group_m = 8;
        a.xcd_remap = 0;
        if (g.scale_only) {
            // 64 x 64 tile of C = beta*C
            const TileCoord tc = map_tile(local, a.tiles_m, a.tiles_n, 8, 0);
            for (int e = threadIdx.x; e < 64 * 64; e += 256) {
                const int i = tc.tm * 64 + e / 64, j = tc.tn * 64 + e % 64;
                if (i < a.M && j < a.N) {
                    float* p = a.C + (int64_t)i * a.ldc + j;
                    *p = (a.beta != 0.f) ? a.beta * *p : 0.f;
                }
            }
        } else {
            switch (g.cfg) {
                case 0: run_tile<typename G::C0>(a, local, lds); break;
                case 1: run_tile<typename G::C1>(a, local, lds); break;
                case 2: run_tile<typename G::C2>(a, local, lds); break;
                default: run_tile<typename G::C3>(a, local, lds); break;
            }
        }
        __syncthreads();  // the next tile's packing reuses the LDS
    }
}

namespace {

struct Plan {
    std::vector<uint64_t> key;
    uint64_t dims = 0;  // dims_key of the set
    int dtype = 0;
    int count = 0;   // problems with at least one tile
    int total = 0;   // tiles
    int grid = 0;
    GroupDesc* d_desc = nullptr;
    int* d_prefix = nullptr;
    int device = -1;
};

std::mutex g_plan_mu;
std::map<uint64_t, Plan> g_plans;

uint64_t fnv(const std::vector<uint64_t>& v)
{
    uint64_t h = 1469598103934665603ull;
    for (uint64_t x : v)
        for (int b = 0; b < 8; ++b) {
            h ^= (x >> (8 * b)) & 0xff;
            h *= 1099511628211ull;
        }
    return h;
}

uint64_t fbits(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return u;
}

// Default threshold: 128 x 128 macro-tiles once both output dimensions fill
// most of one (fewer, more efficient tiles); 64 x 64 otherwise (less padding).
constexpr int kDefaultThreshold = 96;
// Thresholds the tuner times; the last one means "64 x 64 everywhere".
constexpr int kThresholds[] = {0, 64, 96, 160, 256, 512, INT32_MAX};

int choose_cfg(const GroupDesc& g, bool vec, int threshold)
{
    const bool big = g.M >= threshold && g.N >= threshold;
    return (big ? 2 : 0) + (vec ? 0 : 1);
}

// Tuned thresholds by problem-set dimensions (pointers, alpha and beta left out).
std::map<uint64_t, int> g_tuned_threshold;

int build_plan(int64_t count, const int64_t* M, const int64_t* N, const int64_t* K,
               const float* alpha, const void* const* A, const int64_t* lda, const void* const* B,
               const int64_t* ldb, const float* beta, float* const* C, const int64_t* ldc, int dtype,
               int threshold, Plan* plan)
{
    std::vector<GroupDesc> descs;
    for (int64_t p = 0; p < count; ++p) {
        if (M[p] == 0 || N[p] == 0) continue;
        GroupDesc g;
        std::memset(&g, 0, sizeof(g));
        g.A = A[p];
        g.B = B[p];
        g.C = C[p];
        g.lda = lda[p];
        g.ldb = ldb[p];
        g.ldc = ldc[p];
        g.M = (int)M[p];
        g.N = (int)N[p];
        g.K = (int)K[p];
        g.alpha = alpha[p];
        g.beta = beta[p];
        g.scale_only = (K[p] == 0 || alpha[p] == 0.f) ? 1 : 0;
        g.cfg = g.scale_only ? 0 : choose_cfg(g, vec_ok(A[p], lda[p], B[p], ldb[p], dtype), threshold);
        const int t = kGroupTile[g.cfg];
        g.tiles_m = (int)((M[p] + t - 1) / t);
        g.tiles_n = (int)((N[p] + t - 1) / t);
        descs.push_back(g);
    }
    // heaviest tiles first
    std::stable_sort(descs.begin(), descs.end(), [](const GroupDesc& x, const GroupDesc& y) {
        const double wx = x.scale_only ? 0.0 : (double)kGroupTile[x.cfg] * kGroupTile[x.cfg] * x.K;
        const double wy = y.scale_only ? 0.0 : (double)kGroupTile[y.cfg] * kGroupTile[y.cfg] * y.K;
        return wx > wy;
    });
    std::vector<int> prefix(descs.size() + 1, 0);
    for (size_t i = 0; i < descs.size(); ++i) {
        const int64_t tiles = (int64_t)descs[i].tiles_m * descs[i].tiles_n;
        if (prefix[i] + tiles > INT32_MAX) return TGEMM_NOT_SUPPORTED;
        prefix[i + 1] = prefix[i] + (int)tiles;
    }
    plan->dtype = dtype;
    plan->count = (int)descs.size();
    plan->total = prefix.back();
    if (plan->count == 0) return TGEMM_SUCCESS;

    int dev = 0, cus = 256, per_cu = 1;
    (void)hipGetDevice(&dev);
    plan->device = dev;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
    const void* fn = dtype == TGEMM_F32 ? (const void*)&grouped_kernel<MODE_F32>
                                        : (const void*)&grouped_kernel<MODE_X3>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    plan->grid = std::min(plan->total, cus * per_cu);

    if (hipMalloc(&plan->d_desc, descs.size() * sizeof(GroupDesc)) != hipSuccess)
        return TGEMM_ALLOC_FAILED;
    if (hipMalloc(&plan->d_prefix, prefix.size() * sizeof(int)) != hipSuccess) {
        (void)hipFree(plan->d_desc);
        plan->d_desc = nullptr;
        return TGEMM_ALLOC_FAILED;
    }
    if (hipMemcpy(plan->d_desc, descs.data(), descs.size() * sizeof(GroupDesc),
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(plan->d_prefix, prefix.data(), prefix.size() * sizeof(int),
                  hipMemcpyHostToDevice) != hipSuccess)
        return TGEMM_LAUNCH_FAILED;
    return TGEMM_SUCCESS;
}

void free_plan(Plan& p)
{
    if (p.d_desc) (void)hipFree(p.d_desc);
    if (p.d_prefix) (void)hipFree(p.d_prefix);
    p.d_desc = nullptr;
    p.d_prefix = nullptr;
}

int launch_plan(const Plan& p, hipStream_t s)
{
    if (p.count == 0) return TGEMM_SUCCESS;
    if (p.dtype == TGEMM_F32)
        hipLaunchKernelGGL(grouped_kernel<MODE_F32>, dim3(p.grid), dim3(256), 0, s, p.d_desc,
                           p.d_prefix, p.count, p.total);
    else
        hipLaunchKernelGGL(grouped_kernel<MODE_X3>, dim3(p.grid), dim3(256), 0, s, p.d_desc,
                           p.d_prefix, p.count, p.total);
    return hipGetLastError() == hipSuccess ? TGEMM_SUCCESS : TGEMM_LAUNCH_FAILED;
}

int validate_set(int64_t count, const int64_t* M, const int64_t* N, const int64_t* K,
                 const float* alpha, const void* const* A, const int64_t* lda, const void* const* B,
                 const int64_t* ldb, const float* beta, float* const* C, const int64_t* ldc, int dtype)
{
    if (dtype != TGEMM_F32 && dtype != TGEMM_F32_BF16X3) return TGEMM_NOT_SUPPORTED;
    if (count < 0 || count > (1 << 24)) return TGEMM_INVALID_VALUE;
    if (count == 0) return TGEMM_SUCCESS;
    if (!M || !N || !K || !alpha || !A || !lda || !B || !ldb || !beta || !C || !ldc)
        return TGEMM_INVALID_VALUE;
    for (int64_t p = 0; p < count; ++p) {
        const int rc = validate_gemm(M[p], N[p], K[p], alpha[p], A[p], lda[p], B[p], ldb[p], beta[p],
                                     C[p], ldc[p], dtype);
        if (rc != TGEMM_SUCCESS) return rc;
    }
    return TGEMM_SUCCESS;
}

// Key of the dimensions alone: what the tile configuration depends on.
uint64_t dims_key(int64_t count, const int64_t* M, const int64_t* N, const int64_t* K,
                  const float* alpha, const void* const* A, const int64_t* lda, const void* const* B,
                  const int64_t* ldb, int dtype)
{
    std::vector<uint64_t> v;
    v.reserve((size_t)count * 5 + 2);
    v.push_back((uint64_t)count);
    v.push_back((uint64_t)dtype);
    for (int64_t p = 0; p < count; ++p) {
        v.push_back((uint64_t)M[p]);
        v.push_back((uint64_t)N[p]);
        v.push_back((uint64_t)K[p]);
        v.push_back(alpha[p] == 0.f ? 1u : 0u);
        v.push_back(vec_ok(A[p], lda[p], B[p], ldb[p], dtype) ? 1u : 0u);
    }
    return fnv(v);
}

}  // namespace

}  // namespace tg

extern "C" int tgemm_batched(int64_t count, const int64_t* M, const int64_t* N, const int64_t* K,
                             const float* alpha, const void* const* A, const int64_t* lda,
                             const void* const* B, const int64_t* ldb, const float* beta,
                             float* const* C, const int64_t* ldc, int dtype, void* stream)
{
    using namespace tg;
    int rc = validate_set(count, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, dtype);
    if (rc != TGEMM_SUCCESS || count == 0) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);

    // key of the problem set
    std::vector<uint64_t> key;
    key.reserve((size_t)count * 11 + 2);
    key.push_back((uint64_t)count);
    key.push_back((uint64_t)dtype);
    for (int64_t p = 0; p < count; ++p) {
        key.push_back((uint64_t)M[p]);
        key.push_back((uint64_t)N[p]);
        key.push_back((uint64_t)K[p]);
        key.push_back(fbits(alpha[p]));
        key.push_back(fbits(beta[p]));
        key.push_back((uint64_t)(uintptr_t)A[p]);
        key.push_back((uint64_t)(uintptr_t)B[p]);
        key.push_back((uint64_t)(uintptr_t)C[p]);
        key.push_back((uint64_t)lda[p]);
        key.push_back((uint64_t)ldb[p]);
        key.push_back((uint64_t)ldc[p]);
    }
    const uint64_t h = fnv(key);

    std::lock_guard<std::mutex> lk(g_plan_mu);
    int dev = 0;
    (void)hipGetDevice(&dev);
    auto it = g_plans.find(h);
    if (it == g_plans.end() || it->second.key != key || it->second.device != dev) {
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &cap) == hipSuccess && cap != hipStreamCaptureStatusNone)
            return TGEMM_CAPTURE_UNPLANNED;
        rc = ensure_device(s);
        if (rc != TGEMM_SUCCESS) return rc;
        if (it != g_plans.end()) {
            free_plan(it->second);
            g_plans.erase(it);
        }
        const uint64_t dk = dims_key(count, M, N, K, alpha, A, lda, B, ldb, dtype);
        auto tuned = g_tuned_threshold.find(dk);
        const int threshold = tuned != g_tuned_threshold.end() ? tuned->second : kDefaultThreshold;
        Plan plan;
        plan.key = key;
        plan.dims = dk;
        rc = build_plan(count, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, dtype, threshold, &plan);
        if (rc != TGEMM_SUCCESS) {
            free_plan(plan);
            return rc;
        }
        it = g_plans.emplace(h, std::move(plan)).first;
    }
    return launch_plan(it->second, s);
}

extern "C" int tgemm_batched_autotune(int64_t count, const int64_t* M, const int64_t* N,
                                      const int64_t* K, const float* alpha, const void* const* A,
                                      const int64_t* lda, const void* const* B, const int64_t* ldb,
                                      const float* beta, float* const* C, const int64_t* ldc,
                                      int dtype, int reps, void* stream)
{
    using namespace tg;
    if (reps < 1 || reps > 1000) return -TGEMM_INVALID_VALUE;
    int rc = validate_set(count, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, dtype);
    if (rc != TGEMM_SUCCESS) return -rc;
    if (count == 0) return kDefaultThreshold;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) == hipSuccess && cap != hipStreamCaptureStatusNone)
        return -TGEMM_CAPTURE_UNPLANNED;
    rc = ensure_device(s);
    if (rc != TGEMM_SUCCESS) return -rc;

    std::lock_guard<std::mutex> lk(g_plan_mu);
    // The timed launches overwrite C: keep a copy and put it back at the end.
    int64_t total = 0;
    for (int64_t p = 0; p < count; ++p) total += M[p] * N[p];
    float* saved = nullptr;
    if (total > 0 && hipMalloc(&saved, (size_t)total * sizeof(float)) != hipSuccess)
        return -TGEMM_ALLOC_FAILED;
    auto copy_c = [&](bool save) {
        int64_t off = 0;
        for (int64_t p = 0; p < count; ++p) {
            if (M[p] == 0 || N[p] == 0) continue;
            float* packed = saved + off;
            const size_t w = (size_t)N[p] * sizeof(float);
            const hipError_t e =
                save ? hipMemcpy2DAsync(packed, w, C[p], (size_t)ldc[p] * sizeof(float), w, (size_t)M[p],
                                        hipMemcpyDeviceToDevice, s)
                     : hipMemcpy2DAsync(C[p], (size_t)ldc[p] * sizeof(float), packed, w, w, (size_t)M[p],
                                        hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return false;
            off += M[p] * N[p];
        }
        return true;
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    int best = -1;
    float best_ms = 0.f;
    std::vector<std::vector<int>> seen;  // configuration vectors already timed
    rc = copy_c(true) ? TGEMM_SUCCESS : TGEMM_LAUNCH_FAILED;
    for (int threshold : kThresholds) {
        if (rc != TGEMM_SUCCESS) break;
        Plan plan;
        rc = build_plan(count, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, dtype, threshold, &plan);
        if (rc != TGEMM_SUCCESS) {
            free_plan(plan);
            break;
        }
        // thresholds that give the same configuration for every problem are timed once
        std::vector<int> cfgs;
        for (int64_t p = 0; p < count; ++p)
            cfgs.push_back(M[p] >= threshold && N[p] >= threshold ? 1 : 0);
        if (std::find(seen.begin(), seen.end(), cfgs) != seen.end()) {
            free_plan(plan);
            continue;
        }
        seen.push_back(cfgs);
        std::vector<float> times;
        rc = launch_plan(plan, s);  // warm-up
        for (int r = 0; r < reps && rc == TGEMM_SUCCESS; ++r) {
            (void)hipEventRecord(e0, s);
            rc = launch_plan(plan, s);
            (void)hipEventRecord(e1, s);
            if (hipEventSynchronize(e1) != hipSuccess) rc = TGEMM_LAUNCH_FAILED;
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            times.push_back(ms);
        }
        if (hipStreamSynchronize(s) != hipSuccess && rc == TGEMM_SUCCESS) rc = TGEMM_LAUNCH_FAILED;
        free_plan(plan);
        if (rc != TGEMM_SUCCESS) break;
        std::sort(times.begin(), times.end());
        const float med = times[times.size() / 2];
        if (best < 0 || med < best_ms) {
            best = threshold;
            best_ms = med;
        }
    }
    if (rc == TGEMM_SUCCESS && !copy_c(false)) rc = TGEMM_LAUNCH_FAILED;
    if (hipStreamSynchronize(s) != hipSuccess && rc == TGEMM_SUCCESS) rc = TGEMM_LAUNCH_FAILED;
    if (saved) (void)hipFree(saved);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != TGEMM_SUCCESS) return -rc;
    const uint64_t dk = dims_key(count, M, N, K, alpha, A, lda, B, ldb, dtype);
    g_tuned_threshold[dk] = best;
    // plans of these dimensions built before the tuning are rebuilt with the
    // tuned threshold on next use
    for (auto it = g_plans.begin(); it != g_plans.end();) {
        if (it->second.dims == dk) {
            free_plan(it->second);
            it = g_plans.erase(it);
        } else {
            ++it;
        }
    }
    return best;
}

extern "C" void tgemm_shutdown(void)
{
    using namespace tg;
    std::lock_guard<std::mutex> lk(g_plan_mu);
    for (auto& kv : g_plans) free_plan(kv.second);
    g_plans.clear();
    g_tuned_threshold.clear();
    packed_shutdown();
}
