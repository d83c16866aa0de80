// Learned cost model for schedule selection (project addition).  The Tiramisu
// paper (Sections I and II) attributes the shortfall of automatic polyhedral
// schedulers to imprecise machine models and tunes gemm's tile sizes by
// search (Section VI-A); here a small network, trained on the autotuner's own
// measurements, predicts every candidate schedule's runtime so that a
// schedule can be picked without searching.
//
//   features(M, N, K, dtype, schedule, tile order) -> predicted log runtime
//
// Training reads the tuning database, normalises features and targets, and
// runs minibatch Adam with the library's GPU kernels (tgemm_mlp_train_step).
// The weight file holds the network, the normalisation, the training range
// (for the out-of-distribution check), the Adam state and the schedule-table
// hash; a file from another table is refused.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <random>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/tgemm.h"
#include "kargs.h"
#include "registry.h"
#include "select.h"

namespace tg {

int ensure_device(hipStream_t stream);
bool vec_ok(const void* A, int64_t lda, const void* B, int64_t ldb, int dtype);

namespace {

constexpr int kFeatures = 22;
constexpr int kHidden = 256;
constexpr int kLayers = 4;  // 3 hidden layers of 256, one output
const int kDims[kLayers + 1] = {kFeatures, kHidden, kHidden, kHidden, 1};
constexpr uint32_t kMagic = 0x4d434754u;  // "TGCM"
constexpr uint32_t kVersion = 3;
// Tile-order variants the model ranks (the autotuner's set).
const int kVariants[][2] = {{1, 0}, {4, 0}, {8, 0}, {2, 1}, {4, 1}, {8, 1}, {16, 1}, {32, 1}};
// A shape is out of distribution when a log2 dimension lies this far outside
// the training range.
constexpr float kOodMargin = 0.5f;

double lg2(double x) { return std::log2(x > 1.0 ? x : 1.0); }

}  // namespace

// Feature vector of one (problem, schedule, tile order).  Pure host code.
void cost_features(int64_t M, int64_t N, int64_t K, int dtype, const SchedDesc& d, int group_m,
                   int xcd, float* f)
{
    const double tm = (double)((M + d.BM - 1) / d.BM), tn = (double)((N + d.BN - 1) / d.BN);
    const double tiles = tm * tn;
    const double slots = 256.0;
    const double waves = std::ceil(tiles / slots);
    const double kpanels = std::ceil((double)K / d.BK);
    const double flops = 2.0 * M * N * K;
    const double es = dtype == TGEMM_BF16 ? 2.0 : (dtype == TGEMM_FP8_E4M3 ? 1.0 : 4.0);
    const double bytes = es * ((double)M * K + (double)K * N) + 4.0 * M * N;
    int i = 0;
    f[i++] = (float)lg2(M);
    f[i++] = (float)lg2(N);
    f[i++] = (float)lg2(K);
    f[i++] = dtype == TGEMM_F32_BF16X3 ? 1.f : 0.f;
    f[i++] = dtype == TGEMM_BF16 ? 1.f : 0.f;
    f[i++] = dtype == TGEMM_FP8_E4M3 ? 1.f : 0.f;
    f[i++] = (float)lg2(d.BM);
    f[i++] = (float)lg2(d.BN);
    f[i++] = (float)lg2(d.BK);
    f[i++] = d.inplace ? 3.f : d.vec == 4 ? 1.f : (d.vec == 0 ? 2.f : 0.f);  // load width / packed / in-place
    f[i++] = (float)lg2(group_m);
    f[i++] = xcd ? 1.f : 0.f;
    f[i++] = (float)lg2(tiles);
    f[i++] = (float)(tiles / (waves * slots));                     // last-wave occupancy
    f[i++] = (float)(1.0 - (double)M * N / (tiles * d.BM * d.BN)); // padding in partial tiles
    f[i++] = (float)(1.0 - (double)K / (kpanels * d.BK));          // K remainder padding
    f[i++] = (float)lg2(flops);
    f[i++] = (float)lg2(flops / bytes);
    f[i++] = (float)lg2(kpanels);
    f[i++] = (float)d.lds_bytes / (160.f * 1024.f);
    f[i++] = (float)d.split;                                        // stream-K
    f[i++] = d.mfma == 16 ? 1.f : 0.f;                              // 16 x 16 MFMA blocks
}

namespace {

struct Model {
    bool loaded = false;
    uint64_t space = 0;
    float fmean[kFeatures], fstd[kFeatures];
    float ymean = 0.f, ystd = 1.f;
    float lo[3], hi[3];           // training range of log2 M, N, K
    std::vector<float> params;    // host copy
    float* d_params = nullptr;    // device copy
    float* d_work = nullptr;
    float* d_x = nullptr;
    float* d_out = nullptr;
    int cap_rows = 0;
    std::map<std::tuple<int, int64_t, int64_t, int64_t, int>, std::pair<Choice, float>> cache;
};

std::mutex g_cm_mu;
Model g_model;

void free_device(Model& m)
{
    for (float** p : {&m.d_params, &m.d_work, &m.d_x, &m.d_out})
        if (*p) {
            (void)hipFree(*p);
            *p = nullptr;
        }
    m.cap_rows = 0;
}

struct Sample {
    float f[kFeatures];
    float y;  // log(ms)
};

bool parse_num(const char* line, const char* key, double* out)
{
    char pat[48];
    std::snprintf(pat, sizeof(pat), "\"%s\":", key);
    const char* p = std::strstr(line, pat);
    if (!p) return false;
    p += std::strlen(pat);
    while (*p == ' ') ++p;
    char* end = nullptr;
    *out = std::strtod(p, &end);
    return end != p;
}

bool parse_space(const char* line, unsigned long long* out)
{
    const char* p = std::strstr(line, "\"space\": \"");
    if (!p) return false;
    p += std::strlen("\"space\": \"");
    char* end = nullptr;
    *out = std::strtoull(p, &end, 16);
    return end != p;
}

int read_samples(const char* path, std::vector<Sample>* out, float lo[3], float hi[3])
{
    FILE* f = std::fopen(path, "r");
    if (!f) return TGEMM_INVALID_VALUE;
    const unsigned long long space = schedule_space_hash();
    char line[4096];
    for (int i = 0; i < 3; ++i) {
        lo[i] = 1e30f;
        hi[i] = -1e30f;
    }
    while (std::fgets(line, sizeof(line), f)) {
        if (!std::strchr(line, '\n') && !std::feof(f)) {
            int c;
            while ((c = std::fgetc(f)) != EOF && c != '\n') {}
            continue;
        }
        if (!std::strstr(line, "\"valid\": true")) continue;
        unsigned long long h;
        double dt, m, n, k, sid, gm, xcd, ms;
        if (!parse_space(line, &h) || h != space) continue;
        if (!parse_num(line, "dtype", &dt) || !parse_num(line, "M", &m) || !parse_num(line, "N", &n) ||
            !parse_num(line, "K", &k) || !parse_num(line, "sched", &sid) ||
            !parse_num(line, "group_m", &gm) || !parse_num(line, "xcd", &xcd) ||
            !parse_num(line, "ms", &ms))
            continue;
        if (sid < 0 || sid >= num_schedules() || !(ms > 0) || m < 1 || n < 1 || k < 1) continue;
        Sample s;
        cost_features((int64_t)m, (int64_t)n, (int64_t)k, (int)dt, schedule((int)sid), (int)gm,
                      (int)xcd, s.f);
        s.y = (float)std::log(ms);
        out->push_back(s);
        for (int i = 0; i < 3; ++i) {
            lo[i] = std::min(lo[i], s.f[i]);
            hi[i] = std::max(hi[i], s.f[i]);
        }
    }
    std::fclose(f);
    return TGEMM_SUCCESS;
}

template <class T>
bool put(FILE* f, const T* p, size_t n) { return std::fwrite(p, sizeof(T), n, f) == n; }
template <class T>
bool get(FILE* f, T* p, size_t n) { return std::fread(p, sizeof(T), n, f) == n; }

// Weight file: magic, version, space hash, layer count, dims, normalisation,
// training range, parameter count, params, Adam m, Adam v, Adam step.
int save_weights(const char* path, const Model& m, const std::vector<float>& am,
                 const std::vector<float>& av, int64_t step)
{
    FILE* f = std::fopen(path, "wb");
    if (!f) return TGEMM_INVALID_VALUE;
    const uint64_t np = m.params.size();
    const int32_t layers = kLayers;
    bool ok = put(f, &kMagic, 1) && put(f, &kVersion, 1) && put(f, &m.space, 1) &&
              put(f, &layers, 1) && put(f, kDims, kLayers + 1) && put(f, m.fmean, kFeatures) &&
              put(f, m.fstd, kFeatures) && put(f, &m.ymean, 1) && put(f, &m.ystd, 1) &&
              put(f, m.lo, 3) && put(f, m.hi, 3) && put(f, &np, 1) && put(f, m.params.data(), np) &&
              put(f, am.data(), np) && put(f, av.data(), np) && put(f, &step, 1);
    ok = (std::fclose(f) == 0) && ok;
    return ok ? TGEMM_SUCCESS : TGEMM_INTERNAL;
}

int load_weights(const char* path, Model* m)
{
    FILE* f = std::fopen(path, "rb");
    if (!f) return TGEMM_INVALID_VALUE;
    uint32_t magic = 0, version = 0;
    int32_t layers = 0;
    int dims[kLayers + 1];
    uint64_t np = 0;
    bool ok = get(f, &magic, 1) && get(f, &version, 1) && get(f, &m->space, 1) && get(f, &layers, 1);
    ok = ok && magic == kMagic && version == kVersion && layers == kLayers;
    ok = ok && get(f, dims, kLayers + 1) && std::equal(dims, dims + kLayers + 1, kDims);
    ok = ok && get(f, m->fmean, kFeatures) && get(f, m->fstd, kFeatures) && get(f, &m->ymean, 1) &&
         get(f, &m->ystd, 1) && get(f, m->lo, 3) && get(f, m->hi, 3) && get(f, &np, 1);
    ok = ok && np == (uint64_t)tgemm_mlp_param_count(kLayers, kDims);
    if (ok) {
        m->params.resize(np);
        ok = get(f, m->params.data(), np);
    }
    std::fclose(f);
    if (!ok) return TGEMM_INVALID_VALUE;
    if (m->space != schedule_space_hash()) return TGEMM_NOT_SUPPORTED;  // another schedule table
    return TGEMM_SUCCESS;
}

int ensure_capacity(Model& m, int rows)
{
    if (rows <= m.cap_rows && m.d_params) return TGEMM_SUCCESS;
    const int cap = std::max(rows, 256);
    for (float** p : {&m.d_work, &m.d_x, &m.d_out})
        if (*p) {
            (void)hipFree(*p);
            *p = nullptr;
        }
    const int64_t nw = tgemm_mlp_workspace_count(kLayers, kDims, cap);
    if (nw < 0) return TGEMM_INVALID_VALUE;
    if (hipMalloc(&m.d_work, nw * sizeof(float)) != hipSuccess ||
        hipMalloc(&m.d_x, (size_t)cap * kFeatures * sizeof(float)) != hipSuccess ||
        hipMalloc(&m.d_out, (size_t)cap * sizeof(float)) != hipSuccess)
        return TGEMM_ALLOC_FAILED;
    m.cap_rows = cap;
    return TGEMM_SUCCESS;
}

bool in_distribution(const Model& m, int64_t M, int64_t N, int64_t K)
{
    const float q[3] = {(float)lg2(M), (float)lg2(N), (float)lg2(K)};
    for (int i = 0; i < 3; ++i)
        if (q[i] < m.lo[i] - kOodMargin || q[i] > m.hi[i] + kOodMargin) return false;
    return true;
}

// Model argmin over every candidate; caller holds g_cm_mu.  Returns
// TGEMM_NOT_SUPPORTED when there is no model or the shape is out of range.
int predict_locked(int64_t M, int64_t N, int64_t K, int dtype, bool vec_allowed, Choice* out,
                   float* ms_out)
{
    Model& m = g_model;
    if (!m.loaded) return TGEMM_NOT_SUPPORTED;
    if (!in_distribution(m, M, N, K)) return TGEMM_NOT_SUPPORTED;
    const auto key = std::make_tuple(dtype, M, N, K, vec_allowed ? 4 : 1);
    auto it = m.cache.find(key);
    if (it != m.cache.end()) {
        *out = it->second.first;
        if (ms_out) *ms_out = it->second.second;
        return TGEMM_SUCCESS;
    }
    std::vector<float> X;
    std::vector<Choice> cand;
    float f[kFeatures];
    for (int sid = 0; sid < num_schedules(); ++sid) {
        const SchedDesc& d = schedule(sid);
        if (d.dtype != dtype || (d.vec > 1 && !vec_allowed)) continue;
        for (const auto& v : kVariants) {
            cost_features(M, N, K, dtype, d, v[0], v[1], f);
            for (int i = 0; i < kFeatures; ++i) X.push_back((f[i] - m.fmean[i]) / m.fstd[i]);
            cand.push_back(Choice{sid, v[0], v[1]});
        }
    }
    if (cand.empty()) return TGEMM_NOT_SUPPORTED;
    int rc = ensure_device(nullptr);
    if (rc != TGEMM_SUCCESS) return rc;
    const int rows = (int)cand.size();
    if ((rc = ensure_capacity(m, rows)) != TGEMM_SUCCESS) return rc;
    if (hipMemcpy(m.d_x, X.data(), X.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
        return TGEMM_LAUNCH_FAILED;
    rc = tgemm_mlp_forward(kLayers, kDims, m.d_params, rows, m.d_x, m.d_out, m.d_work, nullptr);
    if (rc != TGEMM_SUCCESS) return rc;
    std::vector<float> pred(rows);
    if (hipMemcpy(pred.data(), m.d_out, rows * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
        return TGEMM_LAUNCH_FAILED;
    int best = 0;
    for (int r = 1; r < rows; ++r)
        if (pred[r] < pred[best]) best = r;
    const float ms = std::exp(pred[best] * m.ystd + m.ymean);
    m.cache[key] = std::make_pair(cand[best], ms);
    *out = cand[best];
    if (ms_out) *ms_out = ms;
    return TGEMM_SUCCESS;
}

}  // namespace

// Used by the "model" policy; false when the model cannot answer (no model,
// out of distribution, or a GPU step failed), so the caller falls back.
bool costmodel_choose(int64_t M, int64_t N, int64_t K, int dtype, bool vec_allowed, Choice* out)
{
    std::lock_guard<std::mutex> lk(g_cm_mu);
    return predict_locked(M, N, K, dtype, vec_allowed, out, nullptr) == TGEMM_SUCCESS;
}

bool costmodel_cached(int64_t M, int64_t N, int64_t K, int dtype, bool vec_allowed, Choice* out)
{
    std::lock_guard<std::mutex> lk(g_cm_mu);
    auto it = g_model.cache.find(std::make_tuple(dtype, M, N, K, vec_allowed ? 4 : 1));
    if (it == g_model.cache.end()) return false;
    *out = it->second.first;
    return true;
}

}  // namespace tg

extern "C" {

int tgemm_costmodel_train(const char* db_path, const char* weights_out, int epochs, int batch,
                          float lr, uint64_t seed, float* final_loss)
{
    using namespace tg;
    if (!db_path || !weights_out || epochs < 1 || epochs > 100000 || batch < 1 || batch > 65536 ||
        !(lr > 0.f) || !std::isfinite(lr))
        return TGEMM_INVALID_VALUE;
    std::vector<Sample> data;
    Model m;
    int rc = read_samples(db_path, &data, m.lo, m.hi);
    if (rc != TGEMM_SUCCESS) return rc;
    if (data.size() < 2) return TGEMM_INVALID_VALUE;
    if ((rc = ensure_device(nullptr)) != TGEMM_SUCCESS) return rc;

    // normalisation
    const size_t n = data.size();
    for (int i = 0; i < kFeatures; ++i) {
        double s = 0, s2 = 0;
        for (const Sample& x : data) {
            s += x.f[i];
            s2 += (double)x.f[i] * x.f[i];
        }
        const double mu = s / n, var = std::max(s2 / n - mu * mu, 0.0);
        m.fmean[i] = (float)mu;
        m.fstd[i] = var > 1e-12 ? (float)std::sqrt(var) : 1.f;
    }
    {
        double s = 0, s2 = 0;
        for (const Sample& x : data) {
            s += x.y;
            s2 += (double)x.y * x.y;
        }
        const double mu = s / n, var = std::max(s2 / n - mu * mu, 1e-12);
        m.ymean = (float)mu;
        m.ystd = (float)std::sqrt(var);
    }

    // He-normal initialisation from the seed
    const int64_t np = tgemm_mlp_param_count(kLayers, kDims);
    m.params.assign(np, 0.f);
    std::mt19937_64 rng(seed);
    {
        int64_t off = 0;
        for (int l = 0; l < kLayers; ++l) {
            std::normal_distribution<double> nd(0.0, std::sqrt(2.0 / kDims[l]));
            for (int64_t i = 0; i < (int64_t)kDims[l] * kDims[l + 1]; ++i) m.params[off++] = (float)nd(rng);
            off += kDims[l + 1];  // zero biases
        }
    }
    const int B = (int)std::min<size_t>(batch, n);
    float *d_p = nullptr, *d_g = nullptr, *d_m = nullptr, *d_v = nullptr, *d_x = nullptr,
          *d_y = nullptr, *d_loss = nullptr, *d_work = nullptr;
    const int64_t nw = tgemm_mlp_workspace_count(kLayers, kDims, B);
    bool ok = hipMalloc(&d_p, np * 4) == hipSuccess && hipMalloc(&d_g, np * 4) == hipSuccess &&
              hipMalloc(&d_m, np * 4) == hipSuccess && hipMalloc(&d_v, np * 4) == hipSuccess &&
              hipMalloc(&d_x, n * kFeatures * 4) == hipSuccess && hipMalloc(&d_y, n * 4) == hipSuccess &&
              hipMalloc(&d_loss, 4) == hipSuccess && hipMalloc(&d_work, nw * 4) == hipSuccess;
    std::vector<float> hx(n * kFeatures), hy(n);
    std::vector<size_t> order(n);
    for (size_t i = 0; i < n; ++i) order[i] = i;
    int64_t step = 0;
    float last = 0.f;
    if (ok) {
        ok = hipMemcpy(d_p, m.params.data(), np * 4, hipMemcpyHostToDevice) == hipSuccess &&
             hipMemset(d_m, 0, np * 4) == hipSuccess && hipMemset(d_v, 0, np * 4) == hipSuccess;
    }
    for (int e = 0; ok && e < epochs; ++e) {
        std::shuffle(order.begin(), order.end(), rng);
        for (size_t r = 0; r < n; ++r) {
            const Sample& s = data[order[r]];
            for (int i = 0; i < kFeatures; ++i) hx[r * kFeatures + i] = (s.f[i] - m.fmean[i]) / m.fstd[i];
            hy[r] = (s.y - m.ymean) / m.ystd;
        }
        ok = hipMemcpy(d_x, hx.data(), hx.size() * 4, hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(d_y, hy.data(), hy.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
        // learning rate decays linearly to 10% over the run
        const float lr_e = lr * (1.f - 0.9f * (float)e / (float)epochs);
        for (size_t b0 = 0; ok && b0 + B <= n; b0 += B) {
            ++step;
            ok = tgemm_mlp_train_step(kLayers, kDims, d_p, d_g, d_m, d_v, step, lr_e, B,
                                      d_x + b0 * kFeatures, d_y + b0, d_loss, d_work, nullptr) ==
                 TGEMM_SUCCESS;
        }
        if (ok) ok = hipMemcpy(&last, d_loss, 4, hipMemcpyDeviceToHost) == hipSuccess;
    }
    std::vector<float> am(np), av(np);
    if (ok)
        ok = hipMemcpy(m.params.data(), d_p, np * 4, hipMemcpyDeviceToHost) == hipSuccess &&
             hipMemcpy(am.data(), d_m, np * 4, hipMemcpyDeviceToHost) == hipSuccess &&
             hipMemcpy(av.data(), d_v, np * 4, hipMemcpyDeviceToHost) == hipSuccess;
    for (float* p : {d_p, d_g, d_m, d_v, d_x, d_y, d_loss, d_work})
        if (p) (void)hipFree(p);
    if (!ok) return TGEMM_LAUNCH_FAILED;
    m.space = schedule_space_hash();
    if (final_loss) *final_loss = last;
    return save_weights(weights_out, m, am, av, step);
}

int tgemm_costmodel_load(const char* weights_path)
{
    using namespace tg;
    if (!weights_path) return TGEMM_INVALID_VALUE;
    Model fresh;
    int rc = load_weights(weights_path, &fresh);
    if (rc != TGEMM_SUCCESS) return rc;
    if ((rc = ensure_device(nullptr)) != TGEMM_SUCCESS) return rc;
    std::lock_guard<std::mutex> lk(g_cm_mu);
    free_device(g_model);
    g_model = fresh;
    g_model.cache.clear();
    if (hipMalloc(&g_model.d_params, g_model.params.size() * 4) != hipSuccess ||
        hipMemcpy(g_model.d_params, g_model.params.data(), g_model.params.size() * 4,
                  hipMemcpyHostToDevice) != hipSuccess) {
        free_device(g_model);
        g_model.loaded = false;
        return TGEMM_ALLOC_FAILED;
    }
    g_model.loaded = true;
    return TGEMM_SUCCESS;
}

void tgemm_costmodel_unload(void)
{
    using namespace tg;
    std::lock_guard<std::mutex> lk(g_cm_mu);
    free_device(g_model);
    g_model = Model();
}

int tgemm_costmodel_predict(int64_t M, int64_t N, int64_t K, int dtype, int* schedule_id,
                            int* group_m, int* xcd_remap, float* predicted_ms)
{
    using namespace tg;
    if (M < 1 || N < 1 || K < 1 || !schedule_id || !group_m || !xcd_remap) return TGEMM_INVALID_VALUE;
    if (dtype < TGEMM_F32 || dtype > TGEMM_FP8_E4M3) return TGEMM_NOT_SUPPORTED;
    std::lock_guard<std::mutex> lk(g_cm_mu);
    Choice c;
    float ms = 0.f;
    const int rc = predict_locked(M, N, K, dtype, dense_vec_ok(N, K, dtype), &c, &ms);
    if (rc != TGEMM_SUCCESS) return rc;
    *schedule_id = c.id;
    *group_m = c.group_m;
    *xcd_remap = c.xcd_remap;
    if (predicted_ms) *predicted_ms = ms;
    return TGEMM_SUCCESS;
}

int tgemm_costmodel_predict_all(int64_t M, int64_t N, int64_t K, int dtype, int max_rows,
                                int* schedule_id, int* group_m, int* xcd_remap, float* predicted_ms)
{
    using namespace tg;
    if (M < 1 || N < 1 || K < 1 || max_rows < 1 || !schedule_id || !group_m || !xcd_remap ||
        !predicted_ms)
        return -TGEMM_INVALID_VALUE;
    std::lock_guard<std::mutex> lk(g_cm_mu);
    Model& m = g_model;
    if (!m.loaded) return -TGEMM_NOT_SUPPORTED;
    std::vector<float> X;
    int rows = 0;
    float f[kFeatures];
    for (int sid = 0; sid < num_schedules(); ++sid) {
        const SchedDesc& d = schedule(sid);
        if (d.dtype != dtype) continue;
        for (const auto& v : kVariants) {
            if (rows >= max_rows) return -TGEMM_INVALID_VALUE;
            cost_features(M, N, K, dtype, d, v[0], v[1], f);
            for (int i = 0; i < kFeatures; ++i) X.push_back((f[i] - m.fmean[i]) / m.fstd[i]);
            schedule_id[rows] = sid;
            group_m[rows] = v[0];
            xcd_remap[rows] = v[1];
            ++rows;
        }
    }
    if (rows == 0) return 0;
    int rc = ensure_device(nullptr);
    if (rc != TGEMM_SUCCESS) return -rc;
    if ((rc = ensure_capacity(m, rows)) != TGEMM_SUCCESS) return -rc;
    if (hipMemcpy(m.d_x, X.data(), X.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
        return -TGEMM_LAUNCH_FAILED;
    rc = tgemm_mlp_forward(kLayers, kDims, m.d_params, rows, m.d_x, m.d_out, m.d_work, nullptr);
    if (rc != TGEMM_SUCCESS) return -rc;
    std::vector<float> pred(rows);
    if (hipMemcpy(pred.data(), m.d_out, rows * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return -TGEMM_LAUNCH_FAILED;
    for (int r = 0; r < rows; ++r) predicted_ms[r] = std::exp(pred[r] * m.ystd + m.ymean);
    return rows;
}

int tgemm_costmodel_select(int64_t M, int64_t N, int64_t K, int dtype, int reps,
                           const char* db_path, int* schedule_id, int* group_m, int* xcd_remap,
                           int* used_fallback)
{
    using namespace tg;
    if (M < 1 || N < 1 || K < 1 || !schedule_id || !group_m || !xcd_remap || !used_fallback)
        return TGEMM_INVALID_VALUE;
    int rc = tgemm_costmodel_predict(M, N, K, dtype, schedule_id, group_m, xcd_remap, nullptr);
    if (rc == TGEMM_SUCCESS) {
        *used_fallback = 0;
        return rc;
    }
    if (rc != TGEMM_NOT_SUPPORTED) return rc;
    // no model, or a shape outside its training range: exhaustive autotuning
    *used_fallback = 1;
    const int best = tgemm_autotune(M, N, K, dtype, reps, db_path);
    if (best < 0) return -best;
    Choice c;
    if (!lookup_tuned(dtype, M, N, K, 4, &c)) return TGEMM_INTERNAL;
    *schedule_id = c.id;
    *group_m = c.group_m;
    *xcd_remap = c.xcd_remap;
    return TGEMM_SUCCESS;
}

int tgemm_costmodel_features(int64_t M, int64_t N, int64_t K, int dtype, int schedule_id,
                             int group_m, int xcd_remap, float* out)
{
    using namespace tg;
    if (M < 1 || N < 1 || K < 1 || !out || schedule_id < 0 || schedule_id >= num_schedules() ||
        group_m < 1)
        return TGEMM_INVALID_VALUE;
    cost_features(M, N, K, dtype, schedule(schedule_id), group_m, xcd_remap, out);
    return TGEMM_SUCCESS;
}

}  // extern "C"
