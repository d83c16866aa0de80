/*
 * tgemm — generalized matrix multiply for AMD MI355X (gfx950).
 *
 *     C = alpha * A * B + beta * C
 *
 * The operation is the gemm problem statement of the Tiramisu paper
 * (Section I).  The kernels apply the transformations that paper lists for
 * gemm: two-level tiling (Sections I and VI-A), array packing into a staging
 * buffer (Section I; here the LDS), register blocking (Sections I and VI-A;
 * here MFMA accumulator tiles), separation of full tiles from partial tiles
 * (Section V-A, code generation: full tiles take an unpredicated body, partial
 * tiles a predicated one, so no thread diverges), and tile sizes chosen by
 * measurement (Section VI-A, autotuning).
 *
 * Conventions shared by every entry point
 *   - Row-major storage, no transposes: A is M x K with row stride lda (in
 *     elements), B is K x N with row stride ldb, C is M x N with row stride
 *     ldc.  C is always float32.  The paper fixes none of this; it is the
 *     reading this library takes.
 *   - Matrix and scale pointers are DEVICE pointers owned by the caller; the
 *     library keeps none of them after returning (except tgemm_batched, see
 *     there).  Array arguments of tgemm_batched are HOST arrays.
 *   - `stream` is a hipStream_t passed as void*; NULL is the null stream.
 *     Every call is stream-ordered and returns without synchronising.
 *   - Arguments are validated on the host before any HIP call.  Degenerate
 *     cases follow reference BLAS: M == 0 or N == 0 launches nothing;
 *     K == 0 or alpha == 0 gives C = beta*C without reading A or B;
 *     beta == 0 writes C without reading it (NaN/Inf in the old C vanish).
 *   - Return value: a tgemm_status code.  Faults inside a kernel surface at
 *     the caller's next synchronisation, not here.
 *   - Calls are thread-safe; overlapping calls on one stream are ordered by
 *     the stream, calls on different streams that write the same C race.
 *   - Workspaces the library owns (packing buffers, contraction copies) are
 *     per (device, stream).  One outgrown by a later, larger call is retired,
 *     not freed, and every buffer is kept until tgemm_shutdown(), so a HIP
 *     graph captured over a call stays valid after later eager calls.  Such a
 *     graph writes the workspace of the stream it was captured on: replaying
 *     it on another stream while calls run on the capture stream races.
 */
#ifndef TGEMM_H
#define TGEMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Element type of A and B (C is always float32). */
typedef enum {
    TGEMM_F32 = 0,        /* float32 inputs, float32 MFMA                          */
    TGEMM_F32_BF16X3 = 1, /* float32 inputs; each value split into hi = RNE_bf16(a)
                             and lo = RNE_bf16(a - hi); the product is
                             hi*hi + hi*lo + lo*hi on bf16 MFMA, float32 accumulate */
    TGEMM_BF16 = 2,       /* bfloat16 inputs (uint16 bit patterns)                  */
    TGEMM_FP8_E4M3 = 3    /* OCP E4M3FN bytes (largest finite 448)                  */
} tgemm_dtype;

typedef enum {
    TGEMM_SUCCESS = 0,
    TGEMM_INVALID_VALUE = 1,    /* bad size, leading dimension or null pointer     */
    TGEMM_NOT_SUPPORTED = 2,    /* unknown dtype or schedule                       */
    TGEMM_LAUNCH_FAILED = 3,    /* a HIP call or kernel launch returned an error   */
    TGEMM_ALLOC_FAILED = 4,     /* device memory for a plan could not be allocated */
    TGEMM_CAPTURE_UNPLANNED = 5,/* batched call under stream capture with no plan  */
    TGEMM_INTERNAL = 6,
    TGEMM_NO_DEVICE = 7,        /* no usable gfx950 device                         */
    TGEMM_SCRATCH_TOO_SMALL = 8 /* tgemm_noalloc: the problem's workspace exceeds
                                   TGEMM_NOALLOC_SCRATCH_BYTES                      */
} tgemm_status;

/*
 * Single gemm: C = alpha*A*B + beta*C  (Tiramisu paper, Section I).
 * dtype: TGEMM_F32 or TGEMM_F32_BF16X3 with float* A and B; TGEMM_BF16 or
 * TGEMM_FP8_E4M3 with unscaled low-precision inputs (scale 1).
 * Requires lda >= max(1,K), ldb >= max(1,N), ldc >= max(1,N).
 * The tile schedule comes from the policy (tgemm_set_policy).
 */
int tgemm(int64_t M, int64_t N, int64_t K, float alpha,
          const void* A, int64_t lda, const void* B, int64_t ldb,
          float beta, float* C, int64_t ldc, int dtype, void* stream);

/* Size of the static device array that tgemm_noalloc uses as its workspace. */
#define TGEMM_NOALLOC_SCRATCH_BYTES (128u << 20)

/*
 * tgemm that allocates nothing, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  Arguments, results and degenerate cases as tgemm, with the
 * same schedule choice except that the cost model is never run (its cached
 * answers, the tuning database and the built-in rule are used) and that a
 * stream-K choice, whose per-tile counters the library allocates, runs as its
 * whole-tile schedule (the same tiles and K panels, one workgroup per tile:
 * another summation order, so the result may differ from tgemm's in the last
 * bits; on exact-integer inputs both are exact).  A packed
 * schedule's packing workspace is a static device array of
 * TGEMM_NOALLOC_SCRATCH_BYTES (128 MiB) in the library's code object, one per
 * device, held from the library's first use on that device until the process
 * ends; its device address is looked up once per device, on the first call.
 * No hipMalloc, hipFree or allocating library routine is called.
 * Workspace need of a packed schedule: (Mp + Np) * Kp * e bytes with Mp, Np
 * the sizes rounded up to 256, Kp = K rounded up to 128 (plus 512 bytes per
 * row when that row is a multiple of 4 KB), e = 4 for F32 and
 * F32_BF16X3, 2 for BF16, 1 for FP8_E4M3: 4096 x 4096 x 2048 fits in every
 * form; larger packed problems return TGEMM_SCRATCH_TOO_SMALL before any
 * launch.  Every call on a device shares that device's array: calls that may
 * overlap on one device (different streams, or threads without ordering)
 * race, and must be serialised by the caller.  Each call writes every byte of
 * the region it reads before reading it, so no clearing is needed.
 */
int tgemm_noalloc(int64_t M, int64_t N, int64_t K, float alpha,
                  const void* A, int64_t lda, const void* B, int64_t ldb,
                  float beta, float* C, int64_t ldc, int dtype, void* stream);

/*
 * Same as tgemm with an explicit schedule id (see tgemm_schedule_count /
 * tgemm_schedule_info) and tile-order parameters: group_m >= 1 is the number
 * of tile rows swept together, xcd_remap != 0 gives each XCD a contiguous
 * run of tiles.  Used by the autotuner and by tests that must pin a schedule.
 * Returns TGEMM_NOT_SUPPORTED if the schedule does not serve this dtype or
 * this alignment (vectorised schedules need 16-byte aligned A/B bases and
 * lda, ldb that are multiples of 4 elements).
 */
int tgemm_with_schedule(int64_t M, int64_t N, int64_t K, float alpha,
                        const void* A, int64_t lda, const void* B, int64_t ldb,
                        float beta, float* C, int64_t ldc, int dtype,
                        int schedule_id, int group_m, int xcd_remap, void* stream);

/*
 * Scaled low-precision gemm (project addition; not in the paper):
 *   C = alpha * sum_kb sA[i/128, kb] * sB[kb, j/128] * (sum_{k in kb} qA[i,k] qB[k,j])
 *       + beta * C
 * with one float32 scale per 128 x 128 tile of A (grid ceil(M/128) x
 * ceil(K/128), row-major, row stride ceil(K/128)) and of B (grid
 * ceil(K/128) x ceil(N/128), row stride ceil(N/128)); the last tiles may be
 * partial.  dtype: TGEMM_BF16 (A, B are uint16 bf16 patterns) or
 * TGEMM_FP8_E4M3 (A, B are bytes).  scaleA and scaleB are device pointers and
 * must not be NULL when A and B are read.  Scales must be positive normal
 * floats (packed schedules keep the running sum divided by the current scale
 * product).
 */
int tgemm_scaled(int64_t M, int64_t N, int64_t K, float alpha,
                 const void* A, int64_t lda, const float* scaleA,
                 const void* B, int64_t ldb, const float* scaleB,
                 float beta, float* C, int64_t ldc, int dtype, void* stream);

/*
 * Per-tile quantiser (project addition; not in the paper).  X is a rows x
 * cols float32 row-major device matrix with row stride ldx.  For each
 * 128 x 128 tile (the last ones partial): amax = max |x|;
 *   TGEMM_FP8_E4M3: s = the power of two with amax / s in (224, 448]
 *                   (exponent clamped to [-126, 127]; s = 1 if amax == 0),
 *                   q = round-to-nearest-even, saturating E4M3FN of x/s;
 *   TGEMM_BF16:     s = 2^ceil(log2(amax)) (s = 1 if amax == 0),
 *                   q = round-to-nearest-even bf16 of x/s.
 * Q (device, element size 1 or 2 bytes, row stride ldq) and S (device,
 * ceil(rows/128) x ceil(cols/128), row-major) are written.
 */
int tgemm_quantize_tiles(int64_t rows, int64_t cols, const float* X, int64_t ldx,
                         void* Q, int64_t ldq, float* S, int dtype, void* stream);

/*
 * Grouped gemm over `count` independent problems in one persistent launch
 * (project addition).  Every array argument is a HOST array of length count;
 * the matrix pointers in them are device pointers.  The first call for a new
 * problem set (dimensions, leading dimensions, pointers, alpha, beta, dtype)
 * assigns each problem a tile class by the set's plan shape (below), builds
 * the tile index space and uploads a descriptor table to device memory owned
 * by the library; later calls with
 * the same set launch at most five kernels (packing pass, packed-class
 * tiles, in-place 128 x 128 tiles, in-place 64 x 64 tiles, direct tiles; see
 * tgemm_batched_with_shape for the classes).  The plan shape is what
 * tgemm_batched_autotune measured for sets
 * of these dimensions, else threshold 96 and no packed class.  A plan with packed
 * problems owns a workspace of 4 bytes per element of their A and B (rows
 * padded to 256, K to a multiple of 32) until tgemm_shutdown.
 * If `stream` is capturing and the set has
 * no plan yet, the call returns TGEMM_CAPTURE_UNPLANNED: call once outside
 * capture first.  dtype: TGEMM_F32 or TGEMM_F32_BF16X3.
 */
int tgemm_batched(int64_t count, const int64_t* M, const int64_t* N, const int64_t* K,
                  const float* alpha, const void* const* A, const int64_t* lda,
                  const void* const* B, const int64_t* ldb, const float* beta,
                  float* const* C, const int64_t* ldc, int dtype, void* stream);

/*
 * 3x3 convolution layer as an implicit gemm (project addition; the paper's
 * Conv benchmark layer, Section VI-A, which builds convolutions on sgemm):
 *   Y[n, y, x, co] = alpha * sum_{dy, dx, ci} Xpad[n, y + dy, x + dx, ci] * Wt[dy, dx, ci, co]
 *                    + beta * Y[n, y, x, co]
 * with stride 1 and zero padding 1 (Xpad: X with a border of zeros), so Y
 * has X's height and width.  Layouts (all DEVICE pointers, dense):
 *   X  batch x H x W x Cin (NHWC) float, 16-byte aligned;
 *   Wt 3 x 3 x Cin x Cout float (a 9*Cin x Cout row-major matrix);
 *   Y  batch x H x W x Cout (NHWC) float.
 * The im2col matrix (batch*H*W x 9*Cin) is never formed: tiles read their
 * input pixels directly.  dtype: TGEMM_F32 or TGEMM_F32_BF16X3 (the x3 form
 * of every product).  Cin must be a multiple of 4 (f32) or 8 (x3) and X
 * 16-byte aligned, else TGEMM_NOT_SUPPORTED; sizes beyond 32-bit indexing
 * (batch*H*W, 9*Cin, Cout) give TGEMM_NOT_SUPPORTED.  Degenerate cases as for
 * tgemm: batch, H, W or Cout == 0 is a no-op; Cin == 0 or alpha == 0 gives
 * Y = beta*Y without reading X or Wt; beta == 0 does not read Y.
 * Kernel: the packed one (TGEMM_CONV_PACKED below) when X spans fewer than
 * 2^31 bytes (x3: 2^30 elements), else the direct one; under stream capture
 * with a workspace too small, the direct one.  Packed tile shape: 0 for f32;
 * for x3, 1 (256 x 256) when Cout >= 256 and ceil(M/256)*ceil(Cout/256) >=
 * 256 with M = batch*H*W, else 0.
 */
int tgemm_conv3x3(int64_t batch, int64_t H, int64_t W, int64_t Cin, int64_t Cout, float alpha,
                  const float* X, const float* Wt, float beta, float* Y, int dtype, void* stream);

/* Activations of tgemm_gemm2. */
#define TGEMM_ACT_NONE 0
#define TGEMM_ACT_RELU 1

/*
 * Back-to-back gemm with the intermediate kept on chip (project addition; the
 * paper's VGG block fuses its two layers so that the intermediate stays close
 * to the arithmetic, Section VI-A):
 *   T = act(A B)               A: M x K (lda), B: K x N1 (ldb)
 *   E = alpha * T D + beta * E  D: N1 x N2 (ldd), E: M x N2 (lde)
 * act: TGEMM_ACT_NONE or TGEMM_ACT_RELU (max(x, 0), NaN kept).  All matrices
 * row-major float, DEVICE pointers, any alignment.  T is formed in FP32, 64
 * rows at a time, in LDS and never written to memory.  dtype: TGEMM_F32 or
 * TGEMM_F32_BF16X3 (the x3 form of both products; T is split like any
 * operand).  N1 <= 256, and 64*lda*4, 16*ldb*4 and 16*ldd*4 below 2^31, else
 * TGEMM_NOT_SUPPORTED; lda < K, ldb < N1, ldd < N2 or lde < N2 give
 * TGEMM_INVALID_VALUE.  Degenerate cases as for tgemm: M or N2 == 0 is a no-op;
 * K, N1 or alpha == 0 gives E = beta*E without reading A, B, D; beta == 0 does
 * not read E.
 */
int tgemm_gemm2(int64_t M, int64_t N1, int64_t N2, int64_t K, float alpha, const float* A, int64_t lda,
                const float* B, int64_t ldb, int act, const float* D, int64_t ldd, float beta, float* E,
                int64_t lde, int dtype, void* stream);

/*
 * Binary tensor contraction over labelled modes (project addition; the
 * paper's Baryon benchmark is a dense tensor contraction, Section VI-A):
 *   C[modes_c] = alpha * sum A[modes_a] * B[modes_b] + beta * C[modes_c]
 * summed over the modes of A and B that C does not have.  Each tensor is
 * dense and row-major (its last mode contiguous), float, a DEVICE pointer;
 * n* modes (0 to 8) with integer labels modes_* and extents extents_* (host
 * arrays).  A mode in A, B and C is a batch mode, in A and C a row mode, in
 * B and C a column mode, in A and B a contracted mode.  The contraction runs
 * as a batch of row x contracted by contracted x column gemms (tgemm for one,
 * tgemm_batched_strided for several; dtype TGEMM_F32 or TGEMM_F32_BF16X3); an
 * operand not already laid out [batch, row, contracted] ([batch, contracted,
 * column] for B, [batch, row, column] for C; batch, row and column modes in
 * C's order, contracted modes in A's) is first copied into that order in a
 * per-(device, stream) workspace the library owns (not grown under stream
 * capture: TGEMM_CAPTURE_UNPLANNED).  Returns TGEMM_INVALID_VALUE for a
 * negative extent, a mode twice in one tensor or one label with two
 * extents; TGEMM_NOT_SUPPORTED for more than 8 modes, a mode in only one
 * tensor, or more than 2^24 batch elements.  Empty C is a no-op; no
 * contracted element or alpha == 0 gives C = beta*C without reading A or B.
 */
int tgemm_contract(int na, const int* modes_a, const int64_t* extents_a, const float* A, int nb,
                   const int* modes_b, const int64_t* extents_b, const float* B, int nc, const int* modes_c,
                   const int64_t* extents_c, float* C, float alpha, float beta, int dtype, void* stream);

/*
 * Matrix-core throughput probe (project addition; for stating achieved
 * throughput against a measured peak as well as the datasheet one): launches
 * 2048 workgroups of 4 waves, each wave running `iters` rounds of four
 * independent MFMAs (F32 32x32x2, BF16 32x32x16 or FP8_E4M3 32x32x64) and
 * writing one float per wave to `sink` (DEVICE, at least 8192 floats).
 * *flops (host, may be NULL) receives the algorithmic flops of the launch;
 * the caller times it.  TGEMM_NOT_SUPPORTED for other dtypes,
 * TGEMM_INVALID_VALUE for iters < 0 or a short sink.
 */
int tgemm_mfma_loop(int dtype, int64_t iters, float* sink, int64_t sink_len, double* flops, void* stream);

/* Kernels of tgemm_conv3x3_path. */
#define TGEMM_CONV_AUTO 0   /* as tgemm_conv3x3 */
#define TGEMM_CONV_DIRECT 1 /* A units loaded into registers straight from X; no workspace */
#define TGEMM_CONV_PACKED 2 /* + i: packed tile shape i of the dtype (tgemm_conv3x3_packed_shape) */
#define TGEMM_CONV_RUNTIME_R 0x100 /* or-ed in: the kernel that takes the filter size at run time, also for 3 x 3 */

/*
 * tgemm_conv3x3 with the kernel chosen by the caller (project addition).
 * TGEMM_CONV_DIRECT: the gemm tile body with register-staged loads, each
 * 16-byte unit of the im2col matrix read from its input pixel (zero in the
 * padding).  TGEMM_CONV_PACKED + i: the filter is packed once into a
 * library-owned workspace of K-contiguous rows (array packing, Section I;
 * x3 also splits X into bf16 high and low parts there), and an LDS pipeline
 * brings A panels in with per-lane buffer loads from the input pixels.  The
 * workspace is the per-(device, stream) one of tgemm; it is not grown under
 * stream capture (TGEMM_CAPTURE_UNPLANNED).  Returns TGEMM_INVALID_VALUE for
 * an unknown path and TGEMM_NOT_SUPPORTED when the packed kernel cannot
 * address the problem (X or one 256-row block of packed filter rows of
 * 2^31 bytes or more); otherwise as tgemm_conv3x3.
 */
int tgemm_conv3x3_path(int64_t batch, int64_t H, int64_t W, int64_t Cin, int64_t Cout, float alpha,
                       const float* X, const float* Wt, float beta, float* Y, int dtype, int path,
                       void* stream);

/*
 * R x R convolution layer (R odd, at most 31; the paper's Conv benchmark names
 * 3, 5, 7, 9 and 11): as tgemm_conv3x3_path with Wt R x R x Cin x Cout and
 * zero padding R / 2, so that Y keeps X's height and width; K = R*R*Cin.
 * Kernels are specialised for R = 3 at compile time; other sizes (and 3 x 3
 * with TGEMM_CONV_RUNTIME_R or-ed into `path`) take R at run time.
 * TGEMM_INVALID_VALUE for an even R or R outside [1, 31]; otherwise as
 * tgemm_conv3x3_path.
 */
int tgemm_conv2d(int64_t batch, int64_t H, int64_t W, int64_t Cin, int64_t Cout, int64_t R, float alpha,
                 const float* X, const float* Wt, float beta, float* Y, int dtype, int path, void* stream);

/*
 * Macro-tile (bm x bn), K panel (bk) and LDS pipeline depth (stages) of packed
 * conv tile shape i for dtype (host pointers; any may be NULL).  No HIP call.
 * TGEMM_INVALID_VALUE past the last shape or for a dtype without one.
 */
int tgemm_conv3x3_packed_shape(int dtype, int i, int* bm, int* bn, int* bk, int* stages);

/*
 * tgemm_batched with the plan shape fixed by the caller instead of tuned or
 * defaulted (project addition).  Problems whose M and N both reach `large`
 * (>= 0; INT32_MAX: none) take the packed path: a packing pass copies their A
 * and B^T into a plan-owned workspace (K-contiguous, zero-padded; array
 * packing, Section I) and 256 x 256 macro-tiles stream K panels from it into
 * LDS.  The other problems take 128 x 128 macro-tiles when M and N both reach
 * `threshold` (>= 0; INT32_MAX: 64 x 64 everywhere), 64 x 64 otherwise, with
 * A and B read from the caller's matrices: K panels straight into LDS
 * (in-place tiles; 16-byte loads where rows are 16-byte aligned and K and N
 * are multiples of 4, else 4-byte loads), or, for problems whose tile rows
 * exceed the 2^31-byte reach of a buffer offset, register-staged direct
 * tiles.  ratio > 0 replaces the threshold by a per-problem choice: a
 * problem takes 128 x 128 tiles when ratio * (its number of 128 x 128 tiles)
 * < 1000 * (its number of 64 x 64 tiles), i.e. when the 128 x 128 tiling
 * costs it less if one such tile costs ratio / 1000 times a 64 x 64 tile.
 * Plans are cached per shape.  Returns TGEMM_INVALID_VALUE for a negative
 * threshold or large, or ratio outside [0, 10^6]; otherwise as tgemm_batched.
 */
int tgemm_batched_with_shape(int64_t count, const int64_t* M, const int64_t* N, const int64_t* K,
                             const float* alpha, const void* const* A, const int64_t* lda,
                             const void* const* B, const int64_t* ldb, const float* beta,
                             float* const* C, const int64_t* ldc, int dtype, int threshold,
                             int large, int ratio, void* stream);

/*
 * tgemm_batched over `count` problems of one shape at fixed element strides
 * (project addition): problem p is C + p*strideC = alpha * (A + p*strideA)
 * (B + p*strideB) + beta * (C + p*strideC), float operands (F32 or x3).
 * The plan is cached under these 17 scalars, so a repeated call costs
 * constant host time whatever the count (tgemm_batched hashes every
 * problem's arguments).  Problems with M and N at most 32 skip the plan: one
 * wave per problem multiplies from registers with FP32 MFMAs (both dtypes).  Problems' C blocks must not overlap (strideC >=
 * (M-1)*ldc + N when count > 1) and strides must be >= 0, else
 * TGEMM_INVALID_VALUE; otherwise as tgemm_batched.
 */
int tgemm_batched_strided(int64_t count, int64_t M, int64_t N, int64_t K, float alpha, const void* A,
                          int64_t lda, int64_t strideA, const void* B, int64_t ldb, int64_t strideB,
                          float beta, float* C, int64_t ldc, int64_t strideC, int dtype, void* stream);

/*
 * Plan-shape autotuner of the grouped launch (project addition; the paper
 * chooses tile sizes by measurement, Section VI-A).  Same arguments as
 * tgemm_batched plus `reps` and three host output pointers.  It times one
 * launch of the whole set for every shape (threshold in {0, 64, 96, 160, 256,
 * 512, never} x large in {256, 512, 1024, never}, as in
 * tgemm_batched_with_shape), then the per-problem rule (no packed class) at
 * the ratio of a least-squares fit of the class costs to those timings (time
 * = c + a64 * sum of 64 x 64 tiles * (K + 32) + a128 * the same over
 * 128 x 128 tiles; ratio = 1000 * a128 / a64) and at ratios 1500, 2000, 2500,
 * 3000 and 3500.  Shapes that give every problem the same tiles are timed once.
 * Each time is the median of `reps` timed launches after one warm-up; the
 * fastest shape is kept for problem sets of these dimensions (M, N, K,
 * alpha == 0 and load width per problem).  Later tgemm_batched calls on
 * such sets use it; cached plans of these dimensions are discarded, so a
 * graph captured over one must be captured again.  C is restored to its
 * contents at entry (the timed launches overwrite it; a device copy of C is
 * allocated for the call).  Synchronises `stream`.  Returns
 * TGEMM_CAPTURE_UNPLANNED while `stream` captures.  On success
 * *threshold_out, *large_out and *ratio_out hold the shape chosen
 * (INT32_MAX: never; ratio 0: the threshold rule).
 * reps in [1, 1000].  Without tuning, tgemm_batched uses threshold 96 and
 * no packed class.
 */
int tgemm_batched_autotune(int64_t count, const int64_t* M, const int64_t* N, const int64_t* K,
                           const float* alpha, const void* const* A, const int64_t* lda,
                           const void* const* B, const int64_t* ldb, const float* beta,
                           float* const* C, const int64_t* ldc, int dtype, int reps, void* stream,
                           int* threshold_out, int* large_out, int* ratio_out);

/* Human-readable name of a status code (static string, never NULL). */
const char* tgemm_status_string(int status);

/*
 * Schedule-selection policy for tgemm (Section VI-A: tile size found by
 * measurement).  "default" (built-in rule), "tuned" (the tuning database,
 * else default), "model" (the loaded cost model's argmin; shapes outside its
 * training range, and new shapes while the stream is being captured, fall back
 * to the tuning database, then to the rule), "force:<id>" (one schedule id for
 * every call it serves).
 * Returns TGEMM_INVALID_VALUE for an unknown policy string.
 */
int tgemm_set_policy(const char* policy);

/* Number of compiled schedules and the parameters of one of them.
 * info receives 11 ints: dtype, BM, BN, BK, waves_m, waves_n, vec, lds_bytes,
 * split, mfma, inplace.
 * vec = 4: 16-byte global loads (16-byte aligned bases, row strides multiple of
 * 16 bytes); vec = 1: 4-byte loads (any alignment); vec = 0: packed operands
 * (a pre-pass copies A and B^T, converted and zero-padded, into a workspace
 * the library owns per device and stream; any alignment).
 * split = 1: stream-K (packed schedules only): one resident wave of
 * workgroups splits the (tile, K panel) iterations evenly; a tile shared by
 * several workgroups is summed, in K order, by the last of them to finish,
 * from partial sums in the stream's workspace (2 * slots * BM * BN floats more)
 * and per-tile counters (4 MiB per device and stream, allocated on first use).
 * split = 0: one workgroup per tile.
 * mfma = 32: the MFMAs compute 32 x 32 output blocks (v_mfma_f32_32x32x2f32,
 * 32x32x16_bf16, 32x32x64_f8f6f4); mfma = 16: 16 x 16 blocks (16x16x4f32,
 * 16x16x32_bf16, 16x16x128_f8f6f4; packed schedules only).
 * inplace = 1 (f32 and x3, vec = 1): no packing pass; each tile's K panels go
 * from the caller's A and B straight into LDS with direct-to-LDS buffer loads
 * (16 bytes at any 4-byte alignment), several workgroups per CU; a problem
 * whose BM rows of A or BK rows of B span 2^31 bytes or more is
 * TGEMM_NOT_SUPPORTED for it (tgemm then takes the rule's direct schedule).
 * Host-only: no HIP call. */
int tgemm_schedule_count(void);
int tgemm_schedule_info(int schedule_id, int* info);

/*
 * Tile placement of one launch, computed on the host exactly as the kernels
 * compute it (no HIP call; used to check that the tiling map of Sections III-C and V is a
 * bijection).  For workgroup w in [0, tiles_m*tiles_n) it writes tile_m[w],
 * tile_n[w] and full[w] (1 when the tile lies inside M x N).
 */
int tgemm_tile_map(int64_t M, int64_t N, int BM, int BN, int group_m, int xcd_remap,
                   int32_t* tile_m, int32_t* tile_n, int32_t* full);

/*
 * Measure every schedule that serves (M, N, K, dtype) on random device
 * inputs the library allocates, median of `reps` timed launches each after
 * warm-up, and append one JSON line per schedule to db_path (created if
 * absent).  Schedules whose result differs from a fixed reference schedule
 * on small-integer inputs are recorded as invalid.  Returns the best
 * schedule id (>= 0) or a negative tgemm_status.
 */
int tgemm_autotune(int64_t M, int64_t N, int64_t K, int dtype, int reps,
                   const char* db_path);

/* Load a tuning database (JSON lines) for the "tuned" policy: keeps the
 * fastest valid record per (dtype, M, N, K, load width).  Lines that do not
 * parse, records marked invalid and records of another schedule table (field
 * "space" != tgemm_schedule_space_hash()) are skipped.  Returns the number of
 * records used, or -TGEMM_INVALID_VALUE if the file cannot be opened.
 * Host-only. */
int tgemm_load_tuning_db(const char* db_path);

/* Hash of the compiled schedule table (the "space" field of tuning records).
 * Host-only. */
uint64_t tgemm_schedule_space_hash(void);

/* Schedule the current policy would pick for a dense problem (row strides K
 * and N, 16-byte aligned bases).  Host-only. */
int tgemm_select_schedule(int64_t M, int64_t N, int64_t K, int dtype,
                          int* schedule_id, int* group_m, int* xcd_remap);

/*
 * Cost-model network primitives (project addition; the Tiramisu paper,
 * Sections I and II, notes that automatic schedulers lack a precise cost
 * model).  A ReLU MLP with `layers` layers of widths dims[0..layers]
 * (host array, dims[layers] == 1): Z_l = A_{l-1} W_l + b_l, A_l = relu(Z_l)
 * except for the last layer.  `params` is one flat FP32 device vector, layer by
 * layer: W_l (dims[l] x dims[l+1], row-major) then b_l.  X is rows x dims[0]
 * row-major on the device; y and out have `rows` entries.  `work` is a device
 * scratch buffer of tgemm_mlp_workspace_count() floats owned by the caller.
 * Matrix products run on this library's F32 gemm (built-in schedule rule).
 */
int64_t tgemm_mlp_param_count(int layers, const int* dims);
int64_t tgemm_mlp_workspace_count(int layers, const int* dims, int64_t rows);
int tgemm_mlp_forward(int layers, const int* dims, const float* params, int64_t rows,
                      const float* X, float* out, float* work, void* stream);
/*
 * One training step on a batch: forward, loss = mean((out - y)^2) written to
 * the device scalar `loss`, gradients by the chain rule into `grads` (same
 * layout as params; the derivative of relu at 0 is 0), then one Adam update
 * (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected with `step` >= 1) of
 * params, adam_m and adam_v.  lr == 0 leaves params unchanged.
 */
int tgemm_mlp_train_step(int layers, const int* dims, float* params, float* grads,
                         float* adam_m, float* adam_v, int64_t step, float lr, int64_t rows,
                         const float* X, const float* y, float* loss, float* work, void* stream);

/* The Adam update of tgemm_mlp_train_step alone, on n parameters. */
int tgemm_adam_step(int64_t n, float* params, const float* grads, float* adam_m, float* adam_v,
                    int64_t step, float lr, void* stream);

/*
 * Learned cost model (project addition).  A 22-feature ReLU MLP (3 hidden
 * layers of 256) predicts the log runtime of (problem, schedule, tile order).
 *
 * tgemm_costmodel_train: reads the valid records of a tuning database written
 *   by tgemm_autotune (records of another schedule table are skipped),
 *   normalises features and targets, trains with minibatch Adam on the GPU
 *   (tgemm_mlp_train_step; `epochs` passes, learning rate decaying linearly
 *   from lr to lr/10, He-normal initialisation from `seed`), and writes the
 *   weight file: network, normalisation, training range, Adam state and the
 *   schedule-table hash.  *final_loss (may be NULL) receives the last batch's
 *   normalised MSE.
 * tgemm_costmodel_load: reads a weight file; TGEMM_NOT_SUPPORTED if it was
 *   trained for another schedule table, TGEMM_INVALID_VALUE if it is not a
 *   weight file of this version.  tgemm_costmodel_unload forgets the model.
 * tgemm_costmodel_predict: argmin of the predicted runtime over every
 *   candidate of a dense problem (row strides K and N, 16-byte aligned bases);
 *   TGEMM_NOT_SUPPORTED without a model or when log2 M, N or K lies more than
 *   0.5 outside the training range.
 * tgemm_costmodel_predict_all: predictions for every candidate of a dtype
 *   (host output arrays of max_rows entries); returns the row count or a
 *   negative status.
 * tgemm_costmodel_select: the prediction when the model can answer, else
 *   exhaustive autotuning (tgemm_autotune with `reps`, appending to db_path);
 *   *used_fallback says which.
 * tgemm_costmodel_features: the feature vector (22 floats, host) of one
 *   candidate.  Host-only.
 */
int tgemm_costmodel_train(const char* db_path, const char* weights_out, int epochs, int batch,
                          float lr, uint64_t seed, float* final_loss);
int tgemm_costmodel_load(const char* weights_path);
void tgemm_costmodel_unload(void);
int tgemm_costmodel_predict(int64_t M, int64_t N, int64_t K, int dtype, int* schedule_id,
                            int* group_m, int* xcd_remap, float* predicted_ms);
int tgemm_costmodel_predict_all(int64_t M, int64_t N, int64_t K, int dtype, int max_rows,
                                int* schedule_id, int* group_m, int* xcd_remap,
                                float* predicted_ms);
int tgemm_costmodel_select(int64_t M, int64_t N, int64_t K, int dtype, int reps,
                           const char* db_path, int* schedule_id, int* group_m, int* xcd_remap,
                           int* used_fallback);
int tgemm_costmodel_features(int64_t M, int64_t N, int64_t K, int dtype, int schedule_id,
                             int group_m, int xcd_remap, float* out);

/* Frees plan caches and workspaces owned by the library. */
void tgemm_shutdown(void);

#ifdef __cplusplus
}
#endif
#endif /* TGEMM_H */
