// Grouped gemm: many independent problems C_p = alpha_p A_p B_p + beta_p C_p
// in one persistent launch (project addition; the Tiramisu paper's sgemm is
// the building block of convolutions, Section VI-A, whose layers are batches
// of uneven gemms).
//
// Plan (host, once per problem set): every problem gets a tile configuration
// (macro-tile size and global-load width): 128 x 128 macro-tiles when both M
// and N reach a threshold, 64 x 64 otherwise.  The threshold, and the choice
// between packed and direct operands (below), are built-in defaults unless
// tgemm_batched_autotune has measured the problem set's dimensions, in which
// case the fastest combination it timed is used.
// Problems are ordered by the work of
// one of their tiles, largest first, and their tile counts are prefix-summed
// into one tile index space; a descriptor table and a tile map (tile ->
// problem, tile within the problem) are
// uploaded to device memory the plan owns.  Launch: grid = the number of
// workgroups the device holds at once; workgroup w takes tiles w, w + grid,
// ... of the index space (heavy tiles first, light ones fill the tail), finds
// each tile's problem with one read of the tile map and runs the
// matching tile body of tile_f32x3.h.  A launch allocates and uploads nothing,
// so it can be captured in a HIP graph once the plan exists.
//
// Packed plans (array packing, Section I): the plan also owns a workspace that
// holds every problem's A and B^T in the packed layout of tile_packed.h, rows
// padded to the problem's tile size and K to whole panels.  A launch then runs
// two packing kernels over all problems (one workgroup row per problem) and a
// persistent kernel whose tiles stream K panels from the workspace into LDS
// with NS-stage direct-to-LDS loads, so small tiles keep several panels in
// flight without registers to stage them.
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
#include "tile_packed.h"

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
    int cfg;         // index into GroupCfgs (or GroupPCfgs for a packed plan)
    int tiles_m, tiles_n;
    int scale_only;  // K == 0 or alpha == 0: C = beta*C; A and B are not read
    // packed plans: the problem's packed A (Mp x Kp) and B^T (Np x Kp) in the
    // plan's workspace (hi and, for x3, lo arrays)
    char* Ap;
    char* Alo;
    char* Bp;
    char* Blo;
    int Mp, Np, Kp;
    int vec_a, vec_b;  // the packing may use vector loads on A / B
    int row_units;     // packing work units of A (256 groups of 8 k each); B^T units follow
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

// Tile configurations of the packed grouped kernel: 64 x 64 and 128 x 128
// macro-tiles, 4 waves, panels of BK with NS LDS stages.
template <int MODE>
struct GroupPCfgs {
    using S = PCfg<MODE, 64, 64, (MODE == MODE_F32) ? 16 : 32, 2, 2, (MODE == MODE_F32) ? 4 : 3>;
    using B = PCfg<MODE, 128, 128, (MODE == MODE_F32) ? 16 : 32, 2, 2, (MODE == MODE_F32) ? 4 : 2>;
    static constexpr int LDS = B::LDS_BYTES > S::LDS_BYTES ? B::LDS_BYTES : S::LDS_BYTES;
    static constexpr int KPAD = 32;  // packed K is a multiple of this (both configs' BK divide it)
    static_assert(KPAD % S::BK == 0 && KPAD % B::BK == 0, "panels tile the padded K");
};

// C = beta*C over one 64 x 64 tile (K == 0 or alpha == 0).
__device__ __forceinline__ void scale_tile(const GroupDesc& g, int local)
{
    const TileCoord tc = map_tile(local, g.tiles_m, g.tiles_n, 8, 0);
    for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
        const int i = tc.tm * 64 + e / 64, j = tc.tn * 64 + e % 64;
        if (i < g.M && j < g.N) {
            float* p = g.C + (int64_t)i * g.ldc + j;
            *p = (g.beta != 0.f) ? g.beta * *p : 0.f;
        }
    }
}

// Packing pre-pass of a packed plan, one launch for every problem: work unit
// u is unit map[u].y of problem map[u].x; a problem's units are its A row
// units (256 groups of 8 k each) and then its 64 x 64 B^T blocks.
template <int MODE>
__global__ void __launch_bounds__(256) grouped_pack_kernel(const GroupDesc* __restrict__ desc,
                                                           const int2* __restrict__ map, int total)
{
    __shared__ float tile[64][65];
    for (int u = blockIdx.x; u < total; u += gridDim.x) {
        const int2 pl = map[u];
        const GroupDesc& g = desc[pl.x];
        const int local = pl.y;
        if (local < g.row_units) {
            // row_units * 256 groups fit in 32 bits (the plan caps work units at 2^31)
            const uint32_t per_row = (uint32_t)g.Kp / 8;
            const uint32_t gi = (uint32_t)local * 256 + threadIdx.x, r = gi / per_row;
            if (gi < (uint32_t)g.Mp * per_row)
                pack_row_group<MODE>(g.A, g.lda, g.M, g.K, g.Ap, g.Alo, g.Kp, (int)r,
                                     (int)(gi - r * per_row) * 8, g.vec_a != 0);
        } else {
            const int b = local - g.row_units, kb = (g.Kp + 63) / 64;
            pack_col_block<MODE>(g.B, g.ldb, g.K, g.N, g.Bp, g.Blo, g.Np, g.Kp, (b / kb) * 64,
                                 (b % kb) * 64, tile, g.vec_b != 0);
        }
    }
}

// BIG: the plan has 128 x 128 tiles.  Without them the kernel needs only the
// 64 x 64 configuration's LDS and registers, and more workgroups fit per CU.
template <int MODE, bool BIG>
__global__ void __launch_bounds__(256, BIG ? 2 : 3) grouped_packed_kernel(const GroupDesc* __restrict__ desc,
                                                                          const int2* __restrict__ map,
                                                                          int total)
{
    using G = GroupPCfgs<MODE>;
    __shared__ __attribute__((aligned(1024))) char lds[BIG ? G::LDS : G::S::LDS_BYTES];
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        const int2 pl = map[t];  // (problem, tile within it)
        const GroupDesc& g = desc[pl.x];
        const int local = pl.y;
        if (g.scale_only) {
            scale_tile(g, local);
        } else {
            PackedArgs a;
            a.A = g.Ap;
            a.Alo = g.Alo;
            a.B = g.Bp;
            a.Blo = g.Blo;
            a.C = g.C;
            a.sA = nullptr;
            a.sB = nullptr;
            a.ldc = g.ldc;
            a.lds_a = 0;
            a.lds_b = 0;
            a.M = g.M;
            a.N = g.N;
            a.K = g.K;
            a.Kp = g.Kp;
            a.alpha = g.alpha;
            a.beta = g.beta;
            a.tiles_m = g.tiles_m;
            a.tiles_n = g.tiles_n;
            a.group_m = 8;
            a.xcd_remap = 0;
            const TileCoord tc = map_tile(local, g.tiles_m, g.tiles_n, 8, 0);
            if (!BIG || g.cfg == 0) packed_tile<typename G::S>(a, tc.tm * 64, tc.tn * 64, lds);
            else packed_tile<typename G::B>(a, tc.tm * 128, tc.tn * 128, lds);
        }
        __syncthreads();  // the next tile's loads reuse the LDS
    }
}

template <int MODE>
__global__ void __launch_bounds__(256) grouped_kernel(const GroupDesc* __restrict__ desc,
                                                      const int2* __restrict__ map, int total)
{
    using G = GroupCfgs<MODE>;
    __shared__ __attribute__((aligned(16))) char lds[G::LDS];
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        const int2 pl = map[t];  // (problem, tile within it)
        const GroupDesc& g = desc[pl.x];
        const int local = pl.y;
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
            scale_tile(g, local);
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
    int2* d_map = nullptr;  // tile -> (problem, tile within it)
    int device = -1;
    // packed plans: the packing workspace and the pre-pass work index space
    bool packed = false;
    bool big = false;  // some problem has 128 x 128 tiles
    char* ws = nullptr;
    int2* d_pack_map = nullptr;  // packing unit -> (problem, unit within it)
    int pack_units = 0, pack_grid = 0;
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

// Plan shape: the 128 x 128 threshold and the packed / direct choice.
struct Shape {
    int threshold;
    bool packed;
};
// Default: 128 x 128 macro-tiles once both output dimensions fill most of one
// (fewer, more efficient tiles), 64 x 64 otherwise (less padding); direct
// operands (on sets of small problems the packing pass costs more than the
// packed tiles save: measured on MI355X for 512 problems in [16, 2048]^3).
constexpr Shape kDefaultShape = {96, false};
// Thresholds the tuner times; the last one means "64 x 64 everywhere".
constexpr int kThresholds[] = {0, 64, 96, 160, 256, 512, INT32_MAX};

bool big_tile(const GroupDesc& g, int threshold) { return g.M >= threshold && g.N >= threshold; }

int choose_cfg(const GroupDesc& g, bool vec, int threshold)
{
    return (big_tile(g, threshold) ? 2 : 0) + (vec ? 0 : 1);
}

// Macro-tile edge of a problem's configuration.
int tile_edge(const GroupDesc& g, bool packed) { return packed ? (g.cfg ? 128 : 64) : kGroupTile[g.cfg]; }

// Tuned plan shapes by problem-set dimensions (pointers, alpha and beta left out).
std::map<uint64_t, Shape> g_tuned_shape;

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Index space of prefix sums -> (owner, index within the owner) per element.
std::vector<int2> expand_map(const std::vector<int>& prefix)
{
    std::vector<int2> map((size_t)prefix.back());
    for (size_t p = 0; p + 1 < prefix.size(); ++p)
        for (int t = prefix[p]; t < prefix[p + 1]; ++t) map[(size_t)t] = make_int2((int)p, t - prefix[p]);
    return map;
}

int build_plan(int64_t count, const int64_t* M, const int64_t* N, const int64_t* K,
               const float* alpha, const void* const* A, const int64_t* lda, const void* const* B,
               const int64_t* ldb, const float* beta, float* const* C, const int64_t* ldc, int dtype,
               Shape shape, Plan* plan)
{
    const int threshold = shape.threshold;
    const bool packed = shape.packed;
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
        if (g.scale_only) g.cfg = 0;
        else if (packed) g.cfg = big_tile(g, threshold) ? 1 : 0;
        else g.cfg = choose_cfg(g, vec_ok(A[p], lda[p], B[p], ldb[p], dtype), threshold);
        const int t = tile_edge(g, packed);
        g.tiles_m = (int)((M[p] + t - 1) / t);
        g.tiles_n = (int)((N[p] + t - 1) / t);
        descs.push_back(g);
    }
    // heaviest tiles first
    std::stable_sort(descs.begin(), descs.end(), [packed](const GroupDesc& x, const GroupDesc& y) {
        const double tx = tile_edge(x, packed), ty = tile_edge(y, packed);
        const double wx = x.scale_only ? 0.0 : tx * tx * x.K;
        const double wy = y.scale_only ? 0.0 : ty * ty * y.K;
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
    plan->packed = packed;
    if (plan->count == 0) return TGEMM_SUCCESS;

    if (packed) {
        // workspace layout: per problem A hi, [A lo,] B^T hi, [B^T lo], each 256-byte aligned
        const int64_t es = 4;  // f32 values, or two bf16 arrays for x3: 4 bytes per element either way
        const int64_t arrays = dtype == TGEMM_F32_BF16X3 ? 2 : 1;
        const int64_t esz = es / arrays;
        int64_t off = 0;
        std::vector<int64_t> offs(descs.size());
        std::vector<int> pack_prefix(descs.size() + 1, 0);
        for (size_t i = 0; i < descs.size(); ++i) {
            GroupDesc& g = descs[i];
            int64_t units = 0;
            if (!g.scale_only) {
                const int t = tile_edge(g, true);
                g.Mp = (int)round_up(g.M, t);
                g.Np = (int)round_up(g.N, t);
                g.Kp = (int)round_up(g.K, GroupPCfgs<MODE_F32>::KPAD);
                g.vec_a = pack_rows_vec(g.A, g.lda, 4);
                g.vec_b = pack_cols_vec(g.B, g.ldb, 4);
                if ((int64_t)g.Mp * (g.Kp / 8) >= ((int64_t)1 << 31)) return TGEMM_NOT_SUPPORTED;
                g.row_units = (int)(((int64_t)g.Mp * (g.Kp / 8) + 255) / 256);
                units = g.row_units + (int64_t)((g.Np + 63) / 64) * ((g.Kp + 63) / 64);
                offs[i] = off;
                off += round_up((int64_t)(g.Mp + g.Np) * g.Kp * es, 256);
            }
            if (pack_prefix[i] + units > INT32_MAX) return TGEMM_NOT_SUPPORTED;
            pack_prefix[i + 1] = pack_prefix[i] + (int)units;
        }
        if (off > 0 && hipMalloc(&plan->ws, (size_t)off) != hipSuccess) return TGEMM_ALLOC_FAILED;
        for (size_t i = 0; i < descs.size(); ++i) {
            GroupDesc& g = descs[i];
            if (g.scale_only) continue;
            char* base = plan->ws + offs[i];
            const int64_t a_bytes = (int64_t)g.Mp * g.Kp * esz, b_bytes = (int64_t)g.Np * g.Kp * esz;
            g.Ap = base;
            g.Alo = arrays == 2 ? base + a_bytes : nullptr;
            g.Bp = base + arrays * a_bytes;
            g.Blo = arrays == 2 ? g.Bp + b_bytes : nullptr;
        }
        plan->pack_units = pack_prefix.back();
        std::vector<int2> pmap = expand_map(pack_prefix);
        if (!pmap.empty()) {
            if (hipMalloc(&plan->d_pack_map, pmap.size() * sizeof(int2)) != hipSuccess)
                return TGEMM_ALLOC_FAILED;
            if (hipMemcpy(plan->d_pack_map, pmap.data(), pmap.size() * sizeof(int2),
                          hipMemcpyHostToDevice) != hipSuccess)
                return TGEMM_LAUNCH_FAILED;
        }
    }

    int dev = 0, cus = 256, per_cu = 1;
    (void)hipGetDevice(&dev);
    plan->device = dev;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
    for (const GroupDesc& g : descs) plan->big = plan->big || (!g.scale_only && g.cfg == 1);
    const void* fn;
    if (packed && plan->big)
        fn = dtype == TGEMM_F32 ? (const void*)&grouped_packed_kernel<MODE_F32, true>
                                : (const void*)&grouped_packed_kernel<MODE_X3, true>;
    else if (packed)
        fn = dtype == TGEMM_F32 ? (const void*)&grouped_packed_kernel<MODE_F32, false>
                                : (const void*)&grouped_packed_kernel<MODE_X3, false>;
    else
        fn = dtype == TGEMM_F32 ? (const void*)&grouped_kernel<MODE_F32>
                                : (const void*)&grouped_kernel<MODE_X3>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    plan->grid = std::min(plan->total, cus * per_cu);
    plan->pack_grid = std::min(plan->pack_units, cus * 8);

    if (hipMalloc(&plan->d_desc, descs.size() * sizeof(GroupDesc)) != hipSuccess)
        return TGEMM_ALLOC_FAILED;
    const std::vector<int2> map = expand_map(prefix);
    if (hipMalloc(&plan->d_map, map.size() * sizeof(int2)) != hipSuccess) {
        (void)hipFree(plan->d_desc);
        plan->d_desc = nullptr;
        return TGEMM_ALLOC_FAILED;
    }
    if (hipMemcpy(plan->d_desc, descs.data(), descs.size() * sizeof(GroupDesc),
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(plan->d_map, map.data(), map.size() * sizeof(int2),
                  hipMemcpyHostToDevice) != hipSuccess)
        return TGEMM_LAUNCH_FAILED;
    return TGEMM_SUCCESS;
}

void free_plan(Plan& p)
{
    if (p.d_desc) (void)hipFree(p.d_desc);
    if (p.d_map) (void)hipFree(p.d_map);
    if (p.ws) (void)hipFree(p.ws);
    if (p.d_pack_map) (void)hipFree(p.d_pack_map);
    p.d_desc = nullptr;
    p.d_map = nullptr;
    p.ws = nullptr;
    p.d_pack_map = nullptr;
}

template <int MODE>
void launch_packed(const Plan& p, hipStream_t s)
{
    if (p.pack_units > 0)
        hipLaunchKernelGGL(grouped_pack_kernel<MODE>, dim3(p.pack_grid), dim3(256), 0, s, p.d_desc,
                           p.d_pack_map, p.pack_units);
    if (p.big)
        hipLaunchKernelGGL((grouped_packed_kernel<MODE, true>), dim3(p.grid), dim3(256), 0, s, p.d_desc,
                           p.d_map, p.total);
    else
        hipLaunchKernelGGL((grouped_packed_kernel<MODE, false>), dim3(p.grid), dim3(256), 0, s, p.d_desc,
                           p.d_map, p.total);
}

int launch_plan(const Plan& p, hipStream_t s)
{
    if (p.count == 0) return TGEMM_SUCCESS;
    if (p.packed) {
        if (p.dtype == TGEMM_F32) launch_packed<MODE_F32>(p, s);
        else launch_packed<MODE_X3>(p, s);
    } else if (p.dtype == TGEMM_F32)
        hipLaunchKernelGGL(grouped_kernel<MODE_F32>, dim3(p.grid), dim3(256), 0, s, p.d_desc,
                           p.d_map, p.total);
    else
        hipLaunchKernelGGL(grouped_kernel<MODE_X3>, dim3(p.grid), dim3(256), 0, s, p.d_desc,
                           p.d_map, p.total);
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

namespace tg {
namespace {

// Plan lookup (or build) and launch; `forced` fixes the plan shape.
int batched_run(int64_t count, const int64_t* M, const int64_t* N, const int64_t* K,
                const float* alpha, const void* const* A, const int64_t* lda, const void* const* B,
                const int64_t* ldb, const float* beta, float* const* C, const int64_t* ldc, int dtype,
                const Shape* forced, hipStream_t s)
{
    int rc = validate_set(count, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, dtype);
    if (rc != TGEMM_SUCCESS || count == 0) return rc;

    // key of the problem set (and of a forced shape)
    std::vector<uint64_t> key;
    key.reserve((size_t)count * 11 + 4);
    key.push_back((uint64_t)count);
    key.push_back((uint64_t)dtype);
    key.push_back(forced ? 1u + (uint64_t)forced->packed : 0u);
    key.push_back(forced ? (uint64_t)(uint32_t)forced->threshold : 0u);
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
        auto tuned = g_tuned_shape.find(dk);
        const Shape shape = forced ? *forced : tuned != g_tuned_shape.end() ? tuned->second : kDefaultShape;
        Plan plan;
        plan.key = key;
        plan.dims = dk;
        rc = build_plan(count, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, dtype, shape, &plan);
        if (rc == TGEMM_ALLOC_FAILED && shape.packed) {
            // no room for the packing workspace: direct operands need none
            free_plan(plan);
            plan = Plan();
            plan.key = key;
            plan.dims = dk;
            rc = build_plan(count, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, dtype,
                            Shape{shape.threshold, false}, &plan);
        }
        if (rc != TGEMM_SUCCESS) {
            free_plan(plan);
            return rc;
        }
        it = g_plans.emplace(h, std::move(plan)).first;
    }
    return launch_plan(it->second, s);
}

}  // namespace
}  // namespace tg

extern "C" int tgemm_batched(int64_t count, const int64_t* M, const int64_t* N, const int64_t* K,
                             const float* alpha, const void* const* A, const int64_t* lda,
                             const void* const* B, const int64_t* ldb, const float* beta,
                             float* const* C, const int64_t* ldc, int dtype, void* stream)
{
    return tg::batched_run(count, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, dtype, nullptr,
                           static_cast<hipStream_t>(stream));
}

extern "C" int tgemm_batched_with_shape(int64_t count, const int64_t* M, const int64_t* N,
                                        const int64_t* K, const float* alpha, const void* const* A,
                                        const int64_t* lda, const void* const* B, const int64_t* ldb,
                                        const float* beta, float* const* C, const int64_t* ldc,
                                        int dtype, int threshold, int packed, void* stream)
{
    if (threshold < 0 || (packed != 0 && packed != 1)) return TGEMM_INVALID_VALUE;
    const tg::Shape shape{threshold, packed != 0};
    return tg::batched_run(count, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, dtype, &shape,
                           static_cast<hipStream_t>(stream));
}

extern "C" int tgemm_batched_autotune(int64_t count, const int64_t* M, const int64_t* N,
                                      const int64_t* K, const float* alpha, const void* const* A,
                                      const int64_t* lda, const void* const* B, const int64_t* ldb,
                                      const float* beta, float* const* C, const int64_t* ldc,
                                      int dtype, int reps, void* stream, int* threshold_out,
                                      int* packed_out)
{
    using namespace tg;
    if (reps < 1 || reps > 1000 || !threshold_out || !packed_out) return TGEMM_INVALID_VALUE;
    int rc = validate_set(count, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, dtype);
    if (rc != TGEMM_SUCCESS) return rc;
    *threshold_out = kDefaultShape.threshold;
    *packed_out = kDefaultShape.packed ? 1 : 0;
    if (count == 0) return TGEMM_SUCCESS;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) == hipSuccess && cap != hipStreamCaptureStatusNone)
        return TGEMM_CAPTURE_UNPLANNED;
    rc = ensure_device(s);
    if (rc != TGEMM_SUCCESS) return rc;

    std::lock_guard<std::mutex> lk(g_plan_mu);
    // The timed launches overwrite C: keep a copy and put it back at the end.
    int64_t total = 0;
    for (int64_t p = 0; p < count; ++p) total += M[p] * N[p];
    float* saved = nullptr;
    if (total > 0 && hipMalloc(&saved, (size_t)total * sizeof(float)) != hipSuccess)
        return TGEMM_ALLOC_FAILED;
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
    bool found = false;
    Shape best = kDefaultShape;
    float best_ms = 0.f;
    std::vector<std::vector<int>> seen;  // configuration vectors already timed
    std::vector<Shape> cands;
    for (int packed = 1; packed >= 0; --packed)
        for (int threshold : kThresholds) cands.push_back(Shape{threshold, packed != 0});
    rc = copy_c(true) ? TGEMM_SUCCESS : TGEMM_LAUNCH_FAILED;
    for (const Shape& cand : cands) {
        if (rc != TGEMM_SUCCESS) break;
        // thresholds that give the same configuration for every problem are timed once
        std::vector<int> cfgs(1, cand.packed ? 1 : 0);
        for (int64_t p = 0; p < count; ++p)
            cfgs.push_back(M[p] >= cand.threshold && N[p] >= cand.threshold ? 1 : 0);
        if (std::find(seen.begin(), seen.end(), cfgs) != seen.end()) continue;
        seen.push_back(cfgs);
        Plan plan;
        rc = build_plan(count, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, dtype, cand, &plan);
        if (rc != TGEMM_SUCCESS) {
            free_plan(plan);
            break;
        }
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
        if (!found || med < best_ms) {
            found = true;
            best = cand;
            best_ms = med;
        }
    }
    if (rc == TGEMM_SUCCESS && !copy_c(false)) rc = TGEMM_LAUNCH_FAILED;
    if (hipStreamSynchronize(s) != hipSuccess && rc == TGEMM_SUCCESS) rc = TGEMM_LAUNCH_FAILED;
    if (saved) (void)hipFree(saved);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != TGEMM_SUCCESS) return rc;
    const uint64_t dk = dims_key(count, M, N, K, alpha, A, lda, B, ldb, dtype);
    g_tuned_shape[dk] = best;
    // plans of these dimensions built before the tuning are rebuilt with the
    // tuned shape on next use
    for (auto it = g_plans.begin(); it != g_plans.end();) {
        if (it->second.dims == dk) {
            free_plan(it->second);
            it = g_plans.erase(it);
        } else {
            ++it;
        }
    }
    *threshold_out = best.threshold;
    *packed_out = best.packed ? 1 : 0;
    return TGEMM_SUCCESS;
}

extern "C" void tgemm_shutdown(void)
{
    using namespace tg;
    std::lock_guard<std::mutex> lk(g_plan_mu);
    for (auto& kv : g_plans) free_plan(kv.second);
    g_plans.clear();
    g_tuned_shape.clear();
    packed_shutdown();
}
