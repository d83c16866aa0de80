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

// Stream-K: the iterations (tile t, K panel p), numbered t * panels + p with
// tiles in the grouped order of map_tile, are split into `grid` contiguous,
// nearly equal ranges, one per workgroup of a single resident wave, so no
// workgroup idles in a last partial wave of tiles.  A tile covered by several
// ranges is summed by whichever of its workgroups finishes last: each writes
// its partial sums to its own slot of `ws` and counts itself in cnt[t]; the
// last one adds the partials in K order (so the result does not depend on
// which workgroup that is) and writes C.  Nothing waits on another workgroup.
// The partials are written and read with device-scope (agent) atomic stores
// and loads, which are coherent across the XCDs' L2 caches on their own; a
// device-scope fence would instead write back and invalidate the whole L2 of
// the XCD, and with it the panels the other tiles there are reading.
struct SkArgs {
    float* ws;   // 2 * grid slots of BM * BN floats: a range's first and last tile
    int* cnt;    // per-tile arrival counts; zero before and after every launch
    int total;   // tiles * panels (< 2^31)
    int grid;    // workgroups; every one has at least one iteration (grid <= total)
    int panels;  // K panels per tile
    int q, r;    // total = q * grid + r: ranges 0 .. r-1 hold q + 1 iterations, the others q
};

__device__ __forceinline__ int sk_begin(const SkArgs& k, int v) { return v * k.q + min(v, k.r); }
// The workgroup whose range holds iteration i.
__device__ __forceinline__ int sk_owner(const SkArgs& k, int i)
{
    const int big = k.r * (k.q + 1);
    return i < big ? i / (k.q + 1) : k.r + (i - big) / k.q;
}

// Cache policy bits of a buffer load (gfx950): sc1, the device-scope policy the
// compiler gives an agent-scope atomic load.
constexpr int kSc1 = 16;

// Epilogue of a stream-K range that covers part of tile t.
template <class CF>
struct SkPartial {
    const PackedArgs& a;
    const SkArgs& k;
    int t, v, m0, n0;
    int* flag;  // LDS word: this workgroup sums the tile

    __device__ __forceinline__ float* slot(int u) const
    {
        const bool first = t == sk_begin(k, u) / k.panels;
        return k.ws + (int64_t)(2 * u + (first ? 0 : 1)) * (CF::BM * CF::BN);
    }

    // Sum r of block (i, j) of this lane in a slot: the 64 lanes of a wave hold
    // 64 consecutive floats, so each (device-scope, 4-byte) store or load of a
    // wave covers 256 contiguous bytes, and sum r + 1 follows 256 bytes later.
    __device__ __forceinline__ static int elem(int wave, int i, int j, int r, int lane)
    {
        return (((wave * CF::TM + i) * CF::TN + j) * CF::AR + r) * 64 + lane;
    }

    template <class SC>
    __device__ __forceinline__ void operator()(typename CF::Acc (&acc)[CF::TM][CF::TN], const SC& sc, int wm0,
                                               int wn0, int lane) const
    {
        asm volatile("" : "+v"(lane));  // keep the slot addresses out of the main loop
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        float* mine = slot(v);
#pragma unroll
        for (int i = 0; i < CF::TM; ++i)
#pragma unroll
            for (int j = 0; j < CF::TN; ++j) {
                const float f = sc(i, j);
#pragma unroll
                for (int r = 0; r < CF::AR; ++r)
                    __hip_atomic_store(mine + elem(wave, i, j, r, lane), f * acc[i][j][r], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            }
        const int u0 = sk_owner(k, t * k.panels), u1 = sk_owner(k, (t + 1) * k.panels - 1);
        __builtin_amdgcn_s_waitcnt(0);  // this thread's partial stores have completed ...
        __syncthreads();                // ... and every thread's: the partial is complete
        if (threadIdx.x == 0) {
            const int last = atomicAdd(&k.cnt[t], 1) == u1 - u0;
            // every range has arrived: the counter is ready for the next launch
            if (last) __hip_atomic_store(&k.cnt[t], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            *flag = last;
        }
        __syncthreads();
        if (!*flag) return;
        // sum every range's partial (this one's included, read back) in K order,
        // FB blocks at a time: for each slot, the loads of all FB blocks go out
        // together (one uniform range per block, the lane's offset, r * 256
        // bytes as the instruction's offset), with the device-scope cache
        // policy of the stores (sc1); then the FB blocks are written to C
        constexpr int NBLK = CF::TM * CF::TN;
        constexpr int FB = (NBLK * CF::AR >= 128 ? 32 : 16) / CF::AR;
        static_assert(FB >= 1 && NBLK % FB == 0, "fix-up chunks cover the wave tile");
#pragma unroll
        for (int b0 = 0; b0 < NBLK; b0 += FB) {
            float s[FB][CF::AR];
#pragma unroll
            for (int q = 0; q < FB; ++q)
#pragma unroll
                for (int r = 0; r < CF::AR; ++r) s[q][r] = 0.f;
            for (int u = u0; u <= u1; ++u) {
                const float* src = slot(u);
                float x[FB][CF::AR];
#pragma unroll
                for (int q = 0; q < FB; ++q) {
                    const int i = (b0 + q) / CF::TN, j = (b0 + q) % CF::TN;
                    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                        const_cast<float*>(src) + elem(wave, i, j, 0, 0), 0, CF::AR * 64 * 4, 0x00020000);
#pragma unroll
                    for (int r = 0; r < CF::AR; ++r)
                        x[q][r] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, lane * 4 + r * 256, 0, kSc1));
                }
#pragma unroll
                for (int q = 0; q < FB; ++q)
#pragma unroll
                    for (int r = 0; r < CF::AR; ++r) s[q][r] += x[q][r];
            }
            write_c<1, FB, CF::AR>(
                a.C, a.ldc, a.M, a.N, a.beta, CF::out_row(0, lane), CF::out_col(lane),
                [&](int, int q, float (&v)[CF::AR]) {
#pragma unroll
                    for (int r = 0; r < CF::AR; ++r) v[r] = a.alpha * s[q][r];
                },
                [&](int, int q, int& r0, int& c0) {
                    r0 = m0 + wm0 + CF::MS * ((b0 + q) / CF::TN);
                    c0 = n0 + wn0 + CF::MS * ((b0 + q) % CF::TN);
                },
                [](int r) { return CF::out_row(r, 0); });
        }
    }
};

template <class CF>
struct SkStore {
    TileStore<CF> whole;
    SkPartial<CF> part;
    bool is_whole;
    template <class SC>
    __device__ __forceinline__ void operator()(typename CF::Acc (&acc)[CF::TM][CF::TN], const SC& sc, int wm0,
                                               int wn0, int lane) const
    {
        if (is_whole) whole(acc, sc, wm0, wn0, lane);
        else part(acc, sc, wm0, wn0, lane);
    }
};

template <class CF>
__global__ void __launch_bounds__(CF::NT, CF::WAVES_PER_EU) packed_sk_kernel(PackedArgs a, SkArgs k)
{
    __shared__ __attribute__((aligned(1024))) char lds[CF::LDS_BYTES];
    __shared__ int flag;
    // the workgroups of one XCD (ids equal mod 8) take consecutive ranges, so
    // the tiles they share panels with meet in that XCD's L2
    const int per_xcd = k.grid / kNumXcd;
    const int v = (k.grid % kNumXcd == 0) ? ((int)blockIdx.x % kNumXcd) * per_xcd + (int)blockIdx.x / kNumXcd
                                          : (int)blockIdx.x;
    const int end = sk_begin(k, v + 1);
    using AL = PackedRowsA<CF>;
    for (int it = sk_begin(k, v); it < end;) {
        const int t = it / k.panels;
        const int pb = it - t * k.panels;
        const int pe = min(k.panels, pb + (end - it));
        const TileCoord tc = map_tile(t, a.tiles_m, a.tiles_n, a.group_m, 0);
        const int m0 = tc.tm * CF::BM, n0 = tc.tn * CF::BN;
        const SkStore<CF> epi{TileStore<CF>{a, m0, n0}, SkPartial<CF>{a, k, t, v, m0, n0, &flag},
                              pb == 0 && pe == k.panels};
        if ((CF::MODE == MODE_BF16 || CF::MODE == MODE_FP8) && a.sA)
            packed_tile_range<CF, AL, PackedRowsB<CF>, PackedOps<CF>, true>(a, m0, n0, lds, typename AL::Geom(),
                                                                            pb, pe - pb, epi);
        else
            packed_tile_range<CF, AL, PackedRowsB<CF>, PackedOps<CF>, false>(a, m0, n0, lds, typename AL::Geom(),
                                                                             pb, pe - pb, epi);
        it += pe - pb;
        __syncthreads();  // every wave is done with the LDS stages (and the flag) before the next tile
    }
}

// ------------------------------------------------------------------ host side
namespace {

struct PSched {
    int dtype, mode, BM, BN, BK, WGM, WGN, lds, threads;
    void (*kernel)(PackedArgs);
    void (*sk_kernel)(PackedArgs, SkArgs);  // stream-K form, or null
    int mfma;                               // MFMA block (32 or 16)
};

#define TG_PSCHED(DT, MODE, BM, BN, BK, WGM, WGN, NS)                                             \
    {DT, MODE, BM, BN, BK, WGM, WGN, PCfg<MODE, BM, BN, BK, WGM, WGN, NS>::LDS_BYTES,              \
     PCfg<MODE, BM, BN, BK, WGM, WGN, NS>::NT, &packed_kernel<PCfg<MODE, BM, BN, BK, WGM, WGN, NS>>, \
     nullptr, 32}
// A schedule that also has a stream-K form (a second registry entry).
#define TG_PSCHED_SK(DT, MODE, BM, BN, BK, WGM, WGN, NS)                                          \
    {DT, MODE, BM, BN, BK, WGM, WGN, PCfg<MODE, BM, BN, BK, WGM, WGN, NS>::LDS_BYTES,              \
     PCfg<MODE, BM, BN, BK, WGM, WGN, NS>::NT, &packed_kernel<PCfg<MODE, BM, BN, BK, WGM, WGN, NS>>, \
     &packed_sk_kernel<PCfg<MODE, BM, BN, BK, WGM, WGN, NS>>, 32}
// A schedule on 16 x 16 MFMA blocks.
#define TG_PSCHED16(DT, MODE, BM, BN, BK, WGM, WGN, NS)                                               \
    {DT, MODE, BM, BN, BK, WGM, WGN, PCfg<MODE, BM, BN, BK, WGM, WGN, NS, 16>::LDS_BYTES,              \
     PCfg<MODE, BM, BN, BK, WGM, WGN, NS, 16>::NT, &packed_kernel<PCfg<MODE, BM, BN, BK, WGM, WGN, NS, 16>>, \
     nullptr, 16}

constexpr PSched kPacked[] = {
    // two workgroups per CU (LDS <= 80 KB), 4 waves each
    TG_PSCHED(TGEMM_F32, MODE_F32, 128, 128, 32, 2, 2, 2),
    TG_PSCHED(TGEMM_F32, MODE_F32, 128, 128, 16, 2, 2, 4),
    // four workgroups per CU (LDS 32 KB): one wave of 128 x 128 tiles covers
    // 1024 tiles, for problems whose tile count falls just past 512
    TG_PSCHED_SK(TGEMM_F32, MODE_F32, 128, 128, 16, 2, 2, 2),
    TG_PSCHED_SK(TGEMM_F32_BF16X3, MODE_X3, 128, 128, 16, 2, 2, 2),
    TG_PSCHED(TGEMM_BF16, MODE_BF16, 128, 128, 32, 2, 2, 2),
    TG_PSCHED(TGEMM_FP8_E4M3, MODE_FP8, 128, 128, 64, 2, 2, 2),
    TG_PSCHED(TGEMM_F32_BF16X3, MODE_X3, 256, 128, 16, 2, 2, 3),
    TG_PSCHED(TGEMM_BF16, MODE_BF16, 256, 128, 32, 2, 2, 3),
    TG_PSCHED(TGEMM_FP8_E4M3, MODE_FP8, 256, 128, 64, 2, 2, 3),
    // two workgroups per CU of 8 waves, each wave 32 x 128 of the tile
    TG_PSCHED_SK(TGEMM_F32, MODE_F32, 128, 256, 16, 4, 2, 3),
    // one workgroup per CU, 8 waves
    TG_PSCHED(TGEMM_F32, MODE_F32, 256, 256, 32, 2, 4, 2),
    TG_PSCHED(TGEMM_F32, MODE_F32, 256, 256, 16, 2, 4, 4),
    TG_PSCHED(TGEMM_F32, MODE_F32, 256, 128, 32, 2, 4, 3),
    TG_PSCHED_SK(TGEMM_F32_BF16X3, MODE_X3, 256, 256, 32, 2, 4, 2),
    TG_PSCHED(TGEMM_F32_BF16X3, MODE_X3, 256, 128, 32, 2, 4, 3),
    TG_PSCHED(TGEMM_F32_BF16X3, MODE_X3, 128, 128, 32, 2, 2, 2),
    TG_PSCHED_SK(TGEMM_BF16, MODE_BF16, 256, 256, 64, 2, 4, 2),
    TG_PSCHED(TGEMM_BF16, MODE_BF16, 256, 256, 32, 2, 4, 4),
    TG_PSCHED(TGEMM_BF16, MODE_BF16, 128, 128, 64, 2, 2, 2),
    TG_PSCHED(TGEMM_FP8_E4M3, MODE_FP8, 256, 256, 128, 2, 4, 2),
    TG_PSCHED_SK(TGEMM_FP8_E4M3, MODE_FP8, 256, 256, 128, 4, 2, 2),
    TG_PSCHED(TGEMM_FP8_E4M3, MODE_FP8, 256, 256, 64, 2, 4, 4),
    TG_PSCHED(TGEMM_FP8_E4M3, MODE_FP8, 128, 128, 128, 2, 2, 2),
    // 16 x 16 MFMA blocks (v_mfma_f32_16x16x4f32, 16x16x32_bf16, 16x16x128_f8f6f4)
    TG_PSCHED16(TGEMM_F32, MODE_F32, 128, 256, 32, 4, 2, 2),
    TG_PSCHED16(TGEMM_F32, MODE_F32, 128, 128, 16, 2, 2, 2),
    TG_PSCHED16(TGEMM_F32, MODE_F32, 256, 256, 32, 2, 4, 2),
    TG_PSCHED16(TGEMM_F32_BF16X3, MODE_X3, 128, 128, 32, 2, 2, 2),
    TG_PSCHED16(TGEMM_F32_BF16X3, MODE_X3, 256, 128, 32, 2, 4, 3),
    TG_PSCHED16(TGEMM_BF16, MODE_BF16, 256, 256, 64, 2, 4, 2),
    TG_PSCHED16(TGEMM_BF16, MODE_BF16, 128, 128, 64, 2, 2, 2),
    TG_PSCHED16(TGEMM_FP8_E4M3, MODE_FP8, 256, 256, 128, 4, 2, 2),
    TG_PSCHED16(TGEMM_FP8_E4M3, MODE_FP8, 128, 128, 128, 2, 2, 2),
};
constexpr int kNumPacked = sizeof(kPacked) / sizeof(kPacked[0]);
constexpr int count_sk()
{
    int n = 0;
    for (const PSched& p : kPacked) n += p.sk_kernel != nullptr;
    return n;
}
constexpr int kNumSk = count_sk();

// Registry entries (kernel pointer unused: packed schedules launch through
// run_packed); vec = 0 marks "packed, any alignment".  Entries kNumPacked ..
// are the stream-K forms, in table order; g_sk_of maps them to their row.
SchedDesc g_packed_desc[kNumPacked + kNumSk];
int g_sk_of[kNumSk > 0 ? kNumSk : 1];
struct DescInit {
    DescInit()
    {
        int n = 0;
        for (int i = 0; i < kNumPacked; ++i) {
            const PSched& p = kPacked[i];
            g_packed_desc[i] = SchedDesc{p.dtype, p.BM, p.BN, p.BK, p.WGM, p.WGN, 0, p.lds, p.threads,
                                         nullptr};
            g_packed_desc[i].mfma = p.mfma;
            if (p.sk_kernel) {
                g_packed_desc[kNumPacked + n] = g_packed_desc[i];
                g_packed_desc[kNumPacked + n].split = 1;
                g_sk_of[n++] = i;
            }
        }
    }
} g_desc_init;

// Stream-K arrival counters, one array per (device, stream), zeroed when it is
// allocated and left zeroed by every launch.  Sized for kSkMaxTiles tiles.
constexpr int kSkMaxTiles = 1 << 20;
std::map<std::pair<int, hipStream_t>, int*> g_skcnt;

__global__ void zero_ints(int* p, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

// Workgroups of one resident wave of a kernel (CUs x occupancy), per device.
int resident_slots(const void* fn, int threads)
{
    static std::mutex mu;
    static std::map<std::pair<int, const void*>, int> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(std::make_pair(dev, fn));
    if (it != cache.end()) return it->second;
    int cus = 256, per_cu = 1;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    cache[std::make_pair(dev, fn)] = cus * per_cu;
    return cus * per_cu;
}

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
    *n = kNumPacked + kNumSk;
    return g_packed_desc;
}

// Bytes of stream-K partial sums for packed schedule `pid` (0 unless it is a
// stream-K form), and the per-stream counter array it needs.
size_t sk_workspace_bytes(int pid)
{
    if (pid < kNumPacked) return 0;
    const PSched& p = kPacked[g_sk_of[pid - kNumPacked]];
    const int slots = resident_slots(reinterpret_cast<const void*>(p.sk_kernel), p.threads);
    return (size_t)2 * slots * p.BM * p.BN * sizeof(float);
}

int sk_counters(hipStream_t s, int** out)
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_ws_mu);
    int*& c = g_skcnt[std::make_pair(dev, s)];
    if (!c) {
        hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &st) == hipSuccess && st != hipStreamCaptureStatusNone)
            return TGEMM_CAPTURE_UNPLANNED;
        if (hipMalloc(&c, (size_t)kSkMaxTiles * sizeof(int)) != hipSuccess) {
            c = nullptr;
            return TGEMM_ALLOC_FAILED;
        }
        hipLaunchKernelGGL(zero_ints, dim3(1024), dim3(256), 0, s, c, kSkMaxTiles);
        if (hipGetLastError() != hipSuccess) return TGEMM_LAUNCH_FAILED;
    }
    *out = c;
    return TGEMM_SUCCESS;
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
    if (it != g_ws.end()) {
        free_workspace(it->second);
        g_ws.erase(it);
    }
    auto ic = g_skcnt.find(std::make_pair(dev, s));
    if (ic != g_skcnt.end()) {
        if (ic->second) (void)hipFree(ic->second);
        g_skcnt.erase(ic);
    }
}

void packed_shutdown()
{
    std::lock_guard<std::mutex> lk(g_ws_mu);
    for (auto& kv : g_ws) free_workspace(kv.second);
    g_ws.clear();
    for (auto& kv : g_skcnt)
        if (kv.second) (void)hipFree(kv.second);
    g_skcnt.clear();
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

// pid < kNumPacked: one workgroup per tile.  pid >= kNumPacked: the stream-K
// form of row g_sk_of[pid - kNumPacked], with its partial sums after the packed
// operands in `ws` and the stream's counters `cnt`.
int run_packed_ws(int pid, int64_t M, int64_t N, int64_t K, float alpha, const void* A, int64_t lda,
                  const float* sA, const void* B, int64_t ldb, const float* sB, float beta, float* C,
                  int64_t ldc, int group_m, int xcd_remap, void* ws, int* cnt, hipStream_t s)
{
    const bool sk = pid >= kNumPacked;
    const PSched& p = kPacked[sk ? g_sk_of[pid - kNumPacked] : pid];
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
    const int tiles = a.tiles_m * a.tiles_n;
    if (sk) {
        SkArgs k;
        k.panels = (int)((K + p.BK - 1) / p.BK);
        const int64_t total = (int64_t)tiles * k.panels;
        if (tiles > kSkMaxTiles || total > INT32_MAX || !cnt) return TGEMM_NOT_SUPPORTED;
        k.total = (int)total;
        const int slots = resident_slots(reinterpret_cast<const void*>(p.sk_kernel), p.threads);
        // whole XCD groups, and at least one iteration per workgroup
        int grid = std::min(slots, k.total);
        if (grid >= kNumXcd) grid -= grid % kNumXcd;
        k.grid = grid;
        k.q = k.total / grid;
        k.r = k.total % grid;
        k.cnt = cnt;
        k.ws = reinterpret_cast<float*>(base + packed_workspace_bytes(M, N, K, p.dtype));
        a.group_m = group_m < 1 ? 1 : group_m;
        hipLaunchKernelGGL(p.sk_kernel, dim3((unsigned)grid), dim3(p.threads), 0, s, a, k);
    } else {
        hipLaunchKernelGGL(p.kernel, dim3((unsigned)tiles), dim3(p.threads), 0, s, a);
    }
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
    const int dtype = g_packed_desc[pid].dtype;
    if (!packed_k_ok(K, dtype)) return TGEMM_NOT_SUPPORTED;
    void* ws = nullptr;
    int* cnt = nullptr;
    int rc = packed_workspace(s, packed_workspace_bytes(M, N, K, dtype) + sk_workspace_bytes(pid), &ws);
    if (rc == TGEMM_SUCCESS && pid >= kNumPacked) rc = sk_counters(s, &cnt);
    if (rc != TGEMM_SUCCESS) return rc;
    return run_packed_ws(pid, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, group_m,
                         xcd_remap, ws, cnt, s);
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
    if (pid < 0) {  // direct and in-place schedules use no workspace
        if (scaled)
            return run_scaled(M, N, K, alpha, A, lda, nullptr, B, ldb, nullptr, beta, C, ldc, dtype, ch.id,
                              ch.group_m, ch.xcd_remap, s);
        rc = run_gemm(ch.id, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ch.group_m, ch.xcd_remap, s);
        // an in-place schedule whose rows lie past the reach of its buffer offsets
        if (rc != TGEMM_NOT_SUPPORTED || !schedule(ch.id).inplace) return rc;
        if ((rc = direct_schedule(M, N, K, dtype, vok, &ch)) != TGEMM_SUCCESS) return rc;
        return run_gemm(ch.id, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ch.group_m, ch.xcd_remap, s);
    }
    if (!packed_k_ok(K, dtype)) return TGEMM_NOT_SUPPORTED;
    if (packed_workspace_bytes(M, N, K, dtype) > (size_t)TGEMM_NOALLOC_SCRATCH_BYTES)
        return TGEMM_SCRATCH_TOO_SMALL;
    void* ws = nullptr;
    if ((rc = scratch_address(&ws)) != TGEMM_SUCCESS) return rc;
    // a stream-K form needs counters the library allocates: its row runs instead,
    // one workgroup per tile (same tiles and panels, another summation order)
    const int row = pid >= kNumPacked ? g_sk_of[pid - kNumPacked] : pid;
    return run_packed_ws(row, M, N, K, alpha, A, lda, nullptr, B, ldb, nullptr, beta, C, ldc, ch.group_m,
                         ch.xcd_remap, ws, nullptr, s);
}
