// Training and inference kernels of the cost model's network (project
// addition; the Tiramisu paper, Sections I and II, points at the lack of a
// precise cost model in automatic schedulers).
//
// A ReLU MLP: Z_l = A_{l-1} W_l + b_l, A_l = relu(Z_l) except for the last
// layer, whose Z is the output; mean squared error loss; gradients by the chain
// rule; Adam.  Parameters are one flat FP32 vector, layer by layer: W_l
// (dims[l] x dims[l+1], row-major) then b_l.  Every matrix product is a call of
// this library's own F32 gemm with the built-in schedule rule; the kernels here
// do the element-wise, reduction and transpose steps around it.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "../../include/tgemm.h"
#include "kargs.h"
#include "registry.h"
#include "select.h"

namespace tg {

int ensure_device(hipStream_t stream);
int run_gemm(int id, int64_t M, int64_t N, int64_t K, float alpha, const void* A, int64_t lda,
             const void* B, int64_t ldb, float beta, float* C, int64_t ldc, int group_m,
             int xcd_remap, hipStream_t stream);
bool vec_ok(const void* A, int64_t lda, const void* B, int64_t ldb, int dtype);

namespace {

constexpr int kMaxLayers = 16;
// Adam constants.  Each float is the nearest float32 to the exact constant;
// 1 - beta is stored separately because 1 - 0.999f is not the nearest float
// to 0.001, and the bias corrections are formed in double from the exact values.
constexpr float kBeta1 = 0.9f, kOneMinusBeta1 = 0.1f;
constexpr float kBeta2 = 0.999f, kOneMinusBeta2 = 0.001f;
constexpr float kEps = 1e-8f;
constexpr double kBeta1d = 0.9, kBeta2d = 0.999;

unsigned blocks_for(int64_t n, int per = 256)
{
    int64_t b = (n + per - 1) / per;
    if (b < 1) b = 1;
    if (b > 8192) b = 8192;
    return (unsigned)b;
}

__global__ void bias_act_kernel(float* Z, int rows, int cols, const float* b, int relu)
{
    const int64_t n = (int64_t)rows * cols;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        float v = Z[i] + b[i % cols];
        if (relu) v = v > 0.f ? v : 0.f;
        Z[i] = v;
    }
}

// dst (cols x rows) = src (rows x cols)^T, 32 x 32 tiles through LDS.
__global__ void transpose_kernel(const float* src, int rows, int cols, float* dst)
{
    __shared__ float tile[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x, ty = threadIdx.y;  // 32 x 8
    for (int k = ty; k < 32; k += 8) {
        const int r = by + k, c = bx + tx;
        if (r < rows && c < cols) tile[k][tx] = src[(int64_t)r * cols + c];
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int r = bx + k, c = by + tx;  // dst row = src column
        if (r < cols && c < rows) dst[(int64_t)r * rows + c] = tile[tx][k];
    }
}

__global__ void relu_mask_kernel(float* dA, const float* A, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        if (!(A[i] > 0.f)) dA[i] = 0.f;
}

// out[j] = sum_i dZ[i, j], one thread per column, rows in order.
__global__ void colsum_kernel(const float* dZ, int rows, int cols, float* out)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= cols) return;
    float s = 0.f;
    for (int i = 0; i < rows; ++i) s += dZ[(int64_t)i * cols + j];
    out[j] = s;
}

// dOut = 2 (out - y) / n; partials[block] = sum of squared differences.
__global__ void __launch_bounds__(256) mse_kernel(const float* out, const float* y, int n,
                                                  float* dout, float* partials)
{
    __shared__ float red[256];
    float s = 0.f;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float d = out[i] - y[i];
        dout[i] = 2.f * d / (float)n;
        s += d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) finish_loss_kernel(const float* partials, int nb, int n,
                                                          float* loss)
{
    __shared__ float red[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < nb; i += 256) s += partials[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0] / (float)n;
}

__global__ void adam_kernel(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                            float c1, float c2)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = kBeta1 * m[i] + kOneMinusBeta1 * gi;
        const float vi = kBeta2 * v[i] + kOneMinusBeta2 * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + kEps);
    }
}

int64_t round64(int64_t n) { return (n + 63) / 64 * 64; }

struct Layout {
    int64_t acts[kMaxLayers];  // offsets of A_0 .. A_{L-1} (the last is the output)
    int64_t dA[2];
    int64_t T;
    int64_t partials;
    int64_t total;
};

bool check_dims(int layers, const int* dims)
{
    if (layers < 1 || layers > kMaxLayers || !dims) return false;
    for (int l = 0; l <= layers; ++l)
        if (dims[l] < 1 || dims[l] > 65536) return false;
    return dims[layers] == 1;
}

Layout layout(int layers, const int* dims, int64_t rows)
{
    Layout L;
    int64_t off = 0, maxd = 1;
    for (int l = 0; l <= layers; ++l) maxd = dims[l] > maxd ? dims[l] : maxd;
    for (int l = 0; l < layers; ++l) {
        L.acts[l] = off;
        off += round64(rows * dims[l + 1]);
    }
    L.dA[0] = off;
    off += round64(rows * maxd);
    L.dA[1] = off;
    off += round64(rows * maxd);
    L.T = off;
    off += round64(rows * maxd > maxd * maxd ? rows * maxd : maxd * maxd);
    L.partials = off;
    off += round64(1024);
    L.total = off;
    return L;
}

int64_t param_offset(const int* dims, int l)
{
    int64_t off = 0;
    for (int i = 0; i < l; ++i) off += (int64_t)dims[i] * dims[i + 1] + dims[i + 1];
    return off;
}

// F32 gemm with the built-in schedule rule (never the user's policy, so that
// the cost model cannot recurse into itself).
int gemm_f32(int64_t M, int64_t N, int64_t K, const float* A, int64_t lda, const float* B,
             int64_t ldb, float* C, int64_t ldc, hipStream_t s)
{
    Choice c;
    int rc = default_schedule(M, N, K, TGEMM_F32, vec_ok(A, lda, B, ldb, TGEMM_F32), &c);
    if (rc != TGEMM_SUCCESS) return rc;
    return run_gemm(c.id, M, N, K, 1.f, A, lda, B, ldb, 0.f, C, ldc, c.group_m, c.xcd_remap, s);
}

int forward_impl(int layers, const int* dims, const float* params, int rows, const float* X,
                 float* work, const Layout& L, float* out_last, hipStream_t s)
{
    const float* in = X;
    for (int l = 0; l < layers; ++l) {
        const float* W = params + param_offset(dims, l);
        const float* b = W + (int64_t)dims[l] * dims[l + 1];
        float* Z = (l == layers - 1 && out_last) ? out_last : work + L.acts[l];
        int rc = gemm_f32(rows, dims[l + 1], dims[l], in, dims[l], W, dims[l + 1], Z, dims[l + 1], s);
        if (rc != TGEMM_SUCCESS) return rc;
        hipLaunchKernelGGL(bias_act_kernel, dim3(blocks_for((int64_t)rows * dims[l + 1])), dim3(256),
                           0, s, Z, rows, dims[l + 1], b, l < layers - 1 ? 1 : 0);
        in = Z;
    }
    return hipGetLastError() == hipSuccess ? TGEMM_SUCCESS : TGEMM_LAUNCH_FAILED;
}

}  // namespace
}  // namespace tg

extern "C" {

int64_t tgemm_mlp_param_count(int layers, const int* dims)
{
    if (!tg::check_dims(layers, dims)) return -TGEMM_INVALID_VALUE;
    return tg::param_offset(dims, layers);
}

int64_t tgemm_mlp_workspace_count(int layers, const int* dims, int64_t rows)
{
    if (!tg::check_dims(layers, dims) || rows < 1 || rows > (1 << 24)) return -TGEMM_INVALID_VALUE;
    return tg::layout(layers, dims, rows).total;
}

int tgemm_mlp_forward(int layers, const int* dims, const float* params, int64_t rows,
                      const float* X, float* out, float* work, void* stream)
{
    using namespace tg;
    if (!check_dims(layers, dims) || rows < 1 || rows > (1 << 24)) return TGEMM_INVALID_VALUE;
    if (!params || !X || !out || !work) return TGEMM_INVALID_VALUE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = ensure_device(s);
    if (rc != TGEMM_SUCCESS) return rc;
    const Layout L = layout(layers, dims, rows);
    return forward_impl(layers, dims, params, (int)rows, X, work, L, out, s);
}

int tgemm_mlp_train_step(int layers, const int* dims, float* params, float* grads, float* adam_m,
                         float* adam_v, int64_t step, float lr, int64_t rows, const float* X,
                         const float* y, float* loss, float* work, void* stream)
{
    using namespace tg;
    if (!check_dims(layers, dims) || rows < 1 || rows > (1 << 24) || step < 1) return TGEMM_INVALID_VALUE;
    if (!params || !grads || !adam_m || !adam_v || !X || !y || !loss || !work) return TGEMM_INVALID_VALUE;
    if (!(lr >= 0.f) || !std::isfinite(lr)) return TGEMM_INVALID_VALUE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = ensure_device(s);
    if (rc != TGEMM_SUCCESS) return rc;
    const int R = (int)rows;
    const Layout L = layout(layers, dims, rows);
    rc = forward_impl(layers, dims, params, R, X, work, L, nullptr, s);
    if (rc != TGEMM_SUCCESS) return rc;

    // loss and dOut
    const int nb = (int)blocks_for(R) > 1024 ? 1024 : (int)blocks_for(R);
    float* dcur = work + L.dA[0];
    float* dnext = work + L.dA[1];
    hipLaunchKernelGGL(mse_kernel, dim3(nb), dim3(256), 0, s, work + L.acts[layers - 1], y, R, dcur,
                       work + L.partials);
    hipLaunchKernelGGL(finish_loss_kernel, dim3(1), dim3(256), 0, s, work + L.partials, nb, R, loss);

    float* T = work + L.T;
    for (int l = layers - 1; l >= 0; --l) {
        const int din = dims[l], dout = dims[l + 1];
        const float* W = params + param_offset(dims, l);
        float* gW = grads + param_offset(dims, l);
        float* gb = gW + (int64_t)din * dout;
        if (l < layers - 1)
            hipLaunchKernelGGL(relu_mask_kernel, dim3(blocks_for((int64_t)R * dout)), dim3(256), 0, s,
                               dcur, work + L.acts[l], (int64_t)R * dout);
        // gW = A_{l-1}^T dZ
        const float* Aprev = l == 0 ? X : work + L.acts[l - 1];
        hipLaunchKernelGGL(transpose_kernel, dim3((din + 31) / 32, (R + 31) / 32), dim3(32, 8), 0, s,
                           Aprev, R, din, T);
        rc = gemm_f32(din, dout, R, T, R, dcur, dout, gW, dout, s);
        if (rc != TGEMM_SUCCESS) return rc;
        hipLaunchKernelGGL(colsum_kernel, dim3((dout + 255) / 256), dim3(256), 0, s, dcur, R, dout, gb);
        if (l > 0) {
            // dA_{l-1} = dZ W^T
            hipLaunchKernelGGL(transpose_kernel, dim3((dout + 31) / 32, (din + 31) / 32), dim3(32, 8),
                               0, s, W, din, dout, T);
            rc = gemm_f32(R, din, dout, dcur, dout, T, din, dnext, din, s);
            if (rc != TGEMM_SUCCESS) return rc;
            float* t = dcur;
            dcur = dnext;
            dnext = t;
        }
    }
    const int64_t np = param_offset(dims, layers);
    const double c1 = 1.0 - std::pow(kBeta1d, (double)step);
    const double c2 = 1.0 - std::pow(kBeta2d, (double)step);
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(np)), dim3(256), 0, s, params, grads, adam_m,
                       adam_v, np, lr, (float)c1, (float)c2);
    return hipGetLastError() == hipSuccess ? TGEMM_SUCCESS : TGEMM_LAUNCH_FAILED;
}

int tgemm_adam_step(int64_t n, float* params, const float* grads, float* adam_m, float* adam_v,
                    int64_t step, float lr, void* stream)
{
    using namespace tg;
    if (n < 0 || step < 1 || !(lr >= 0.f) || !std::isfinite(lr)) return TGEMM_INVALID_VALUE;
    if (n == 0) return TGEMM_SUCCESS;
    if (!params || !grads || !adam_m || !adam_v) return TGEMM_INVALID_VALUE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = ensure_device(s);
    if (rc != TGEMM_SUCCESS) return rc;
    const double c1 = 1.0 - std::pow(kBeta1d, (double)step);
    const double c2 = 1.0 - std::pow(kBeta2d, (double)step);
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n)), dim3(256), 0, s, params, grads, adam_m,
                       adam_v, n, lr, (float)c1, (float)c2);
    return hipGetLastError() == hipSuccess ? TGEMM_SUCCESS : TGEMM_LAUNCH_FAILED;
}

}  // extern "C"
