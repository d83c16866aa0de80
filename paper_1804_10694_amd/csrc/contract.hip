// Binary tensor contraction over labelled modes (project addition; the
// paper's Baryon benchmark is a dense tensor contraction, Section VI-A),
// mapped onto the library's gemm:
//
//   C[modes_c] = alpha * sum_{contracted} A[modes_a] * B[modes_b] + beta * C[modes_c]
//
// Modes are classified as batch (in A, B and C), row (A and C), column (B and
// C) and contracted (A and B).  With batch, row and column modes in C's order
// and contracted modes in A's order, the canonical layouts are
//   A* = [batch, row, contracted], B* = [batch, contracted, column],
//   C* = [batch, row, column],
// i.e. a batch of Mf x Kf by Kf x Nf row-major products.  A tensor already in
// its canonical order is used in place; any other is copied into the
// canonical order by permute_kernel (C is copied back after the products).
// One product runs through tgemm, a batch through the grouped launch
// (tgemm_batched_strided), so the schedule choice, tiling and precision forms
// are those of the gemm paths.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/tgemm.h"
#include "registry.h"

namespace tg {

int ensure_device(hipStream_t stream);

constexpr int kMaxModes = 8;

struct PermArgs {
    int nd;
    int64_t ext[kMaxModes];      // destination extents, row-major
    int64_t sstride[kMaxModes];  // source stride (elements) along each destination dimension
};

// dst (dense, row-major over p.ext) = src read through p.sstride: writes are
// contiguous, reads follow the permutation.
__global__ void __launch_bounds__(256) permute_kernel(const float* __restrict__ src, float* __restrict__ dst,
                                                      int64_t total, PermArgs p)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t rem = i, off = 0;
        for (int d = p.nd - 1; d >= 0; --d) {
            const int64_t c = rem % p.ext[d];
            rem /= p.ext[d];
            off += c * p.sstride[d];
        }
        dst[i] = src[off];
    }
}

__global__ void __launch_bounds__(256) scale_kernel(float* x, int64_t total, float beta)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = beta != 0.f ? beta * x[i] : 0.f;
}

namespace {

unsigned grid_for(int64_t total) { return (unsigned)std::min<int64_t>((total + 255) / 256, 8192); }

// Per (device, stream) workspace of the canonical copies, grown on demand.  An
// outgrown buffer is retired, not freed (a graph captured over an earlier call
// still uses it), and freed at shutdown.
struct CtWorkspace {
    void* ptr = nullptr;
    size_t bytes = 0;
    std::vector<void*> retired;
};
std::mutex g_ct_mu;
std::map<std::pair<int, hipStream_t>, CtWorkspace> g_ct_ws;

int ct_workspace(hipStream_t s, size_t bytes, void** out)
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_ct_mu);
    CtWorkspace& w = g_ct_ws[std::make_pair(dev, s)];
    if (w.bytes < bytes) {
        hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &st) == hipSuccess && st != hipStreamCaptureStatusNone)
            return TGEMM_CAPTURE_UNPLANNED;
        void* p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) return TGEMM_ALLOC_FAILED;
        if (w.ptr) w.retired.push_back(w.ptr);
        w.ptr = p;
        w.bytes = bytes;
    }
    *out = w.ptr;
    return TGEMM_SUCCESS;
}

struct Tensor {
    std::vector<int> modes;
    std::vector<int64_t> ext;
    std::vector<int64_t> stride;  // row-major element strides

    int64_t stride_of(int m) const
    {
        for (size_t d = 0; d < modes.size(); ++d)
            if (modes[d] == m) return stride[d];
        return 0;
    }
    bool has(int m) const { return std::find(modes.begin(), modes.end(), m) != modes.end(); }
};

int make_tensor(int n, const int* modes, const int64_t* ext, Tensor* t)
{
    if (n < 0) return TGEMM_INVALID_VALUE;
    if (n > kMaxModes) return TGEMM_NOT_SUPPORTED;
    if (n > 0 && (!modes || !ext)) return TGEMM_INVALID_VALUE;
    t->modes.assign(modes, modes + n);
    t->ext.assign(ext, ext + n);
    t->stride.assign(n, 1);
    for (int d = 0; d < n; ++d) {
        if (ext[d] < 0) return TGEMM_INVALID_VALUE;
        for (int e = 0; e < d; ++e)
            if (modes[e] == modes[d]) return TGEMM_INVALID_VALUE;  // a mode twice in one tensor
    }
    for (int d = n - 2; d >= 0; --d) t->stride[d] = t->stride[d + 1] * std::max<int64_t>(ext[d + 1], 1);
    return TGEMM_SUCCESS;
}

// Copy `src` (tensor s) into the dense row-major tensor with modes `order`.
int permute_into(const float* src, const Tensor& s, const std::vector<int>& order,
                 const std::map<int, int64_t>& ext, float* dst, hipStream_t st)
{
    PermArgs p{};
    p.nd = (int)order.size();
    int64_t total = 1;
    for (int d = 0; d < p.nd; ++d) {
        p.ext[d] = ext.at(order[d]);
        p.sstride[d] = s.stride_of(order[d]);
        total *= p.ext[d];
    }
    if (p.nd == 0) {
        p.nd = 1;
        p.ext[0] = 1;
        p.sstride[0] = 0;
    }
    if (total == 0) return TGEMM_SUCCESS;
    hipLaunchKernelGGL(permute_kernel, dim3(grid_for(total)), dim3(256), 0, st, src, dst, total, p);
    return hipGetLastError() == hipSuccess ? TGEMM_SUCCESS : TGEMM_LAUNCH_FAILED;
}

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

}  // namespace

void contract_shutdown()
{
    std::lock_guard<std::mutex> lk(g_ct_mu);
    for (auto& kv : g_ct_ws) {
        if (kv.second.ptr) (void)hipFree(kv.second.ptr);
        for (void* p : kv.second.retired) (void)hipFree(p);
    }
    g_ct_ws.clear();
}

}  // namespace tg

extern "C" int tgemm_contract(int na, const int* modes_a, const int64_t* extents_a, const float* A, int nb,
                              const int* modes_b, const int64_t* extents_b, const float* B, int nc,
                              const int* modes_c, const int64_t* extents_c, float* C, float alpha, float beta,
                              int dtype, void* stream)
{
    using namespace tg;
    if (dtype != TGEMM_F32 && dtype != TGEMM_F32_BF16X3) return TGEMM_NOT_SUPPORTED;
    if (!(alpha == alpha) || !(beta == beta)) return TGEMM_INVALID_VALUE;
    Tensor ta, tb, tc;
    int rc;
    if ((rc = make_tensor(na, modes_a, extents_a, &ta)) != TGEMM_SUCCESS) return rc;
    if ((rc = make_tensor(nb, modes_b, extents_b, &tb)) != TGEMM_SUCCESS) return rc;
    if ((rc = make_tensor(nc, modes_c, extents_c, &tc)) != TGEMM_SUCCESS) return rc;
    // one extent per mode label
    std::map<int, int64_t> ext;
    for (const Tensor* t : {&ta, &tb, &tc})
        for (size_t d = 0; d < t->modes.size(); ++d) {
            auto it = ext.find(t->modes[d]);
            if (it != ext.end() && it->second != t->ext[d]) return TGEMM_INVALID_VALUE;
            ext[t->modes[d]] = t->ext[d];
        }
    // every mode appears in exactly two or all three tensors
    for (const auto& kv : ext) {
        const int m = kv.first;
        if ((int)ta.has(m) + (int)tb.has(m) + (int)tc.has(m) < 2) return TGEMM_NOT_SUPPORTED;
    }
    std::vector<int> batch, rows, cols, red;
    for (int m : tc.modes) {
        if (ta.has(m) && tb.has(m)) batch.push_back(m);
        else if (ta.has(m)) rows.push_back(m);
        else cols.push_back(m);
    }
    for (int m : ta.modes)
        if (tb.has(m) && !tc.has(m)) red.push_back(m);
    auto prod = [&](const std::vector<int>& v) {
        int64_t p = 1;
        for (int m : v) {
            const int64_t e = ext[m];
            if (e != 0 && p > INT64_MAX / 4 / e) return (int64_t)-1;  // keeps byte counts in range
            p *= e;
        }
        return p;
    };
    const int64_t Bt = prod(batch), Mf = prod(rows), Nf = prod(cols), Kf = prod(red);
    if (Bt < 0 || Mf < 0 || Nf < 0 || Kf < 0) return TGEMM_NOT_SUPPORTED;
    // element counts of the canonical tensors, in bytes, within int64
    const double lim = 1e18;
    if ((double)Bt * Mf * Nf * 4 > lim || (double)Bt * Mf * Kf * 4 > lim || (double)Bt * Kf * Nf * 4 > lim)
        return TGEMM_NOT_SUPPORTED;
    const int64_t nC = Bt * Mf * Nf;
    if (nC == 0) return TGEMM_SUCCESS;
    if (!C) return TGEMM_INVALID_VALUE;
    const bool reads = alpha != 0.f && Kf > 0;
    if (reads && (!A || !B)) return TGEMM_INVALID_VALUE;
    if (Bt > (1 << 24)) return TGEMM_NOT_SUPPORTED;  // the grouped launch's problem-count limit
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((rc = ensure_device(s)) != TGEMM_SUCCESS) return rc;
    if (!reads) {
        hipLaunchKernelGGL(scale_kernel, dim3(grid_for(nC)), dim3(256), 0, s, C, nC, beta);
        return hipGetLastError() == hipSuccess ? TGEMM_SUCCESS : TGEMM_LAUNCH_FAILED;
    }

    std::vector<int> oa(batch), ob(batch), oc(batch);
    oa.insert(oa.end(), rows.begin(), rows.end());
    oa.insert(oa.end(), red.begin(), red.end());
    ob.insert(ob.end(), red.begin(), red.end());
    ob.insert(ob.end(), cols.begin(), cols.end());
    oc.insert(oc.end(), rows.begin(), rows.end());
    oc.insert(oc.end(), cols.begin(), cols.end());
    const bool copy_a = oa != ta.modes, copy_b = ob != tb.modes, copy_c = oc != tc.modes;
    const int64_t bytes_a = copy_a ? round_up(Bt * Mf * Kf * 4, 256) : 0;
    const int64_t bytes_b = copy_b ? round_up(Bt * Kf * Nf * 4, 256) : 0;
    const int64_t bytes_c = copy_c ? round_up(nC * 4, 256) : 0;
    const float* Ac = A;
    const float* Bc = B;
    float* Cc = C;
    if (bytes_a + bytes_b + bytes_c > 0) {
        void* ws = nullptr;
        if ((rc = ct_workspace(s, (size_t)(bytes_a + bytes_b + bytes_c), &ws)) != TGEMM_SUCCESS) return rc;
        char* w = static_cast<char*>(ws);
        if (copy_a) {
            float* d = reinterpret_cast<float*>(w);
            if ((rc = permute_into(A, ta, oa, ext, d, s)) != TGEMM_SUCCESS) return rc;
            Ac = d;
        }
        if (copy_b) {
            float* d = reinterpret_cast<float*>(w + bytes_a);
            if ((rc = permute_into(B, tb, ob, ext, d, s)) != TGEMM_SUCCESS) return rc;
            Bc = d;
        }
        if (copy_c) {
            Cc = reinterpret_cast<float*>(w + bytes_a + bytes_b);
            if (beta != 0.f && (rc = permute_into(C, tc, oc, ext, Cc, s)) != TGEMM_SUCCESS) return rc;
        }
    }

    if (Bt == 1) {
        rc = tgemm(Mf, Nf, Kf, alpha, Ac, std::max<int64_t>(Kf, 1), Bc, std::max<int64_t>(Nf, 1), beta, Cc,
                   std::max<int64_t>(Nf, 1), dtype, stream);
    } else {
        rc = tgemm_batched_strided(Bt, Mf, Nf, Kf, alpha, Ac, std::max<int64_t>(Kf, 1), Mf * Kf, Bc,
                                   std::max<int64_t>(Nf, 1), Kf * Nf, beta, Cc, std::max<int64_t>(Nf, 1), Mf * Nf,
                                   dtype, stream);
    }
    if (rc != TGEMM_SUCCESS) return rc;
    if (copy_c) {
        // back to C's own mode order: C[modes_c] = C*[oc]
        Tensor tcs;
        tcs.modes = oc;
        tcs.ext.resize(oc.size());
        tcs.stride.assign(oc.size(), 1);
        for (size_t d = 0; d < oc.size(); ++d) tcs.ext[d] = ext[oc[d]];
        for (int d = (int)oc.size() - 2; d >= 0; --d) tcs.stride[d] = tcs.stride[d + 1] * tcs.ext[d + 1];
        if ((rc = permute_into(Cc, tcs, tc.modes, ext, C, s)) != TGEMM_SUCCESS) return rc;
    }
    return TGEMM_SUCCESS;
}
