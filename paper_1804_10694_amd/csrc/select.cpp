// Schedule selection policies and the tuning database reader.
#include "select.h"

#include <algorithm>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "../../include/tgemm.h"
#include "registry.h"

namespace tg {

namespace {

enum Policy { POLICY_DEFAULT = 0, POLICY_TUNED = 1, POLICY_FORCE = 2, POLICY_MODEL = 3 };

struct TunedEntry {
    Choice choice;
    double ms;
};

std::mutex g_sel_mu;
Policy g_policy = POLICY_DEFAULT;
int g_force_id = -1;
std::map<std::tuple<int, int64_t, int64_t, int64_t, int>, TunedEntry> g_tuned;  // (dtype,M,N,K,vec)

bool json_number(const char* line, const char* key, double* out)
{
    char pat[64];
    std::snprintf(pat, sizeof(pat), "\"%s\":", key);
    const char* p = std::strstr(line, pat);
    if (!p) return false;
    p += std::strlen(pat);
    while (*p == ' ') ++p;
    char* end = nullptr;
    const double v = std::strtod(p, &end);
    if (end == p) return false;
    *out = v;
    return true;
}

bool json_true(const char* line, const char* key)
{
    char pat[64];
    std::snprintf(pat, sizeof(pat), "\"%s\": true", key);
    if (std::strstr(line, pat)) return true;
    std::snprintf(pat, sizeof(pat), "\"%s\":true", key);
    return std::strstr(line, pat) != nullptr;
}

bool json_hex(const char* line, const char* key, unsigned long long* out)
{
    char pat[64];
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

void register_locked(int dtype, int64_t M, int64_t N, int64_t K, int vec, const Choice& c, double ms)
{
    const auto key = std::make_tuple(dtype, M, N, K, vec);
    auto it = g_tuned.find(key);
    if (it == g_tuned.end() || ms < it->second.ms) g_tuned[key] = TunedEntry{c, ms};
}

}  // namespace

void register_tuned(int dtype, int64_t M, int64_t N, int64_t K, int vec, const Choice& c, double ms)
{
    std::lock_guard<std::mutex> lk(g_sel_mu);
    register_locked(dtype, M, N, K, vec, c, ms);
}

namespace {
// Fastest tuned record usable with the operands' alignment (16-byte loads
// allowed -> both load widths compete).  Caller holds g_sel_mu.
bool lookup_locked(int dtype, int64_t M, int64_t N, int64_t K, bool vec_allowed, Choice* out)
{
    const TunedEntry* best = nullptr;
    for (int vec : {4, 1, 0}) {  // 0: packed operands, any alignment
        if (vec == 4 && !vec_allowed) continue;
        auto it = g_tuned.find(std::make_tuple(dtype, M, N, K, vec));
        if (it != g_tuned.end() && (!best || it->second.ms < best->ms)) best = &it->second;
    }
    if (!best) return false;
    *out = best->choice;
    return true;
}
}  // namespace

bool lookup_tuned(int dtype, int64_t M, int64_t N, int64_t K, int vec, Choice* out)
{
    std::lock_guard<std::mutex> lk(g_sel_mu);
    return lookup_locked(dtype, M, N, K, vec > 1, out);
}

bool dense_vec_ok(int64_t N, int64_t K, int dtype)
{
    const int64_t es = dtype == TGEMM_BF16 ? 2 : (dtype == TGEMM_FP8_E4M3 ? 1 : 4);
    return (K * es) % 16 == 0 && (N * es) % 16 == 0;
}

int find_schedule(int dtype, int BM, int BN, int BK, int vec, int WGM, int WGN, int lds, int mfma, int split,
                  int inplace)
{
    for (int i = 0; i < num_schedules(); ++i) {
        const SchedDesc& d = schedule(i);
        if (d.dtype == dtype && d.BM == BM && d.BN == BN && d.BK == BK && d.vec == vec &&
            d.WGM == WGM && d.WGN == WGN && (lds < 0 || d.lds_bytes == lds) && d.split == split &&
            d.mfma == mfma && d.inplace == inplace)
            return i;
    }
    return -1;
}

int direct_schedule(int64_t M, int64_t N, int64_t K, int dtype, bool vec_allowed, Choice* out)
{
    (void)K;
    const int vec = vec_allowed ? 4 : 1;
    auto tiles = [&](int bm, int bn) { return ((M + bm - 1) / bm) * ((N + bn - 1) / bn); };
    int id = -1;
    // Measured on MI355X at 8192^3: 128x128 macro-tiles beat 256-wide ones for the
    // direct kernels; 64-wide tiles keep small problems spread over the 256 CUs.
    if (dtype == TGEMM_F32) {
        // rows that 16-byte loads cannot take: 64 x 64 tiles at any size
        if (tiles(128, 128) >= 192 && vec == 4) id = find_schedule(dtype, 128, 128, 32, vec);
        else id = find_schedule(dtype, 64, 64, 16, vec);
    } else if (dtype == TGEMM_F32_BF16X3) {
        if (tiles(128, 128) >= 192 && vec == 4) id = find_schedule(dtype, 128, 128, 32, vec);
        else id = find_schedule(dtype, 64, 64, 32, vec);
    } else if (dtype == TGEMM_BF16) {
        if (tiles(128, 128) >= 192) id = find_schedule(dtype, 128, 128, 64, vec);
        else id = find_schedule(dtype, 64, 64, 64, vec);
    } else if (dtype == TGEMM_FP8_E4M3) {
        if (tiles(256, 128) >= 512) id = find_schedule(dtype, 256, 128, 128, vec);
        else if (tiles(128, 128) >= 192) id = find_schedule(dtype, 128, 128, 128, vec);
        else id = find_schedule(dtype, 64, 128, 128, vec);
    }
    if (id < 0) return TGEMM_NOT_SUPPORTED;
    out->id = id;
    out->group_m = 8;
    out->xcd_remap = 1;
    return TGEMM_SUCCESS;
}

int default_schedule(int64_t M, int64_t N, int64_t K, int dtype, bool vec_allowed, Choice* out)
{
    auto tiles = [&](int bm, int bn) { return ((M + bm - 1) / bm) * ((N + bn - 1) / bn); };
    auto take = [&](int id) {
        out->id = id;
        out->group_m = 8;
        out->xcd_remap = 1;
        return TGEMM_SUCCESS;
    };
    // Large problems take packed operands (the packing pass costs O(MK + KN)
    // against O(MNK)).  Measured on MI355X:
    //  - f32: 128 x 256 macro-tiles of 8 waves (4 x 2, each wave 32 x 128),
    //    three 24 KB LDS stages, two workgroups per CU: 144 TFLOP/s at 8192^3
    //    and 91 at 4097 x 3001 x 2053, against 136 and 83 for 128 x 128 tiles
    //    of 4 waves (64 x 64 each) on the same GPU, and 122 for the best
    //    direct schedule.  The transposed wave shape (128 x 32) gains nothing.
    //    Smaller problems keep the 128 x 128 tiles;
    //  - x3, bf16 and e4m3: 256 x 256 macro-tiles of 8 waves, down to half a
    //    wave of tiles (one workgroup per CU still beats 128 x 128 tiles
    //    there); e4m3 with 128-deep panels and its waves 4 x 2 (64 x 128
    //    each), 1317 TFLOP/s at 16384^3 against 1266 with waves 2 x 4 and
    //    1195 for 128 x 128 tiles of four workgroups per CU (which it takes
    //    below that size).
    //  - f32 with 256 to 383 tiles of 128 x 256 (half to three quarters of a
    //    wave at two workgroups per CU): 128 x 128 tiles on 16 x 16 MFMA blocks,
    //    four workgroups per CU (3000^3: 0.59 ms against 0.73 for 128 x 256).
    //  - f32 and x3 with M or N at most 128 keep the direct tiles (over 2080
    //    shapes log-uniform in [64, 8192], tuned exhaustively on MI355X, the
    //    packed f32 128 x 256 tiles reached 0.33-0.58 of the best schedule
    //    there), and so do rows that 16-byte loads cannot take, on 64 x 64
    //    tiles (rule against the exhaustive optimum on that set, geometric
    //    mean: f32 0.923 -> 0.950, x3 0.915 -> 0.926);
    //  - stream-K (f32 128 x 256, or 128 x 128 below 384 tiles of 128 x 256;
    //    x3 256 x 256) where whole tiles would leave
    //    a large part of the last wave of workgroups idle: f32 when the tiles
    //    fill less than 85% of their waves (4097 x 3001 x 2053: 0.48 ms against
    //    0.57; 3000^3 0.48 against 0.58; 2500 x 1800 x 4000 0.36 against 0.50;
    //    8192^3 and 3500 x 2100 x 1500, at 100% and 93%, keep whole tiles), and
    //    f32 and x3 when too few tiles remain for the packed whole-tile forms
    //    (x3 1024 x 1024 x 8192: 0.14 ms against 0.19); in both cases only with
    //    at least 8 K panels per workgroup of the stream-K wave and enough
    //    tiles (16 and 8) that few workgroups share one.
    const bool narrow = (dtype == TGEMM_F32 || dtype == TGEMM_F32_BF16X3) && (M <= 128 || N <= 128);
    // Deep K on few tiles (K >= 4096, under 768 tiles of 64 x 64, M and N at
    // least 256), f32 and x3 alike: stream-K, which spreads K over every CU
    // (f32 1000^2 x 8192 0.234 ms against 0.248 in place; x3 0.136 against
    // 0.255).
    const bool deep = K >= 4096 && tiles(64, 64) < 768 && std::min(M, N) >= 256 && packed_k_ok(K, dtype);
    if (dtype == TGEMM_F32 && deep) {
        const int sk = tiles(128, 256) >= 16 ? find_schedule(dtype, 128, 256, 16, 0, 4, 2, -1, 32, 1)
                                             : find_schedule(dtype, 128, 128, 16, 0, 2, 2, -1, 32, 1);
        if (sk >= 0) return take(sk);
    }
    // f32 takes in-place tiles except on large squarish problems (at least
    // 2048 tiles of 128 x 256 and M, N > 512), which keep the packed 128 x 256
    // tiles: no packing pass, eight (64 x 64) or four (128 x 128) workgroups
    // per CU; 128 x 128 when its tiles fill at least 60% of waves of 768
    // workgroups (a threshold set by measurement) and M, N >= 256.  Over the
    // 2080 shapes of the cost-model study (exhaustively tuned on MI355X, every
    // schedule and tile order), the best schedule was an in-place one for
    // 1876; this rule (with the deep-K exception) reaches a geometric
    // mean of 0.978 of the exhaustive optimum there, against 0.849 for the
    // rule with the in-place tiles only above 1000 tiles of 64 x 64 and 0.787
    // without them (4097 x 3001 x 2053: 0.57 -> 0.44 ms).
    if (dtype == TGEMM_F32 && (tiles(128, 256) < 2048 || std::min(M, N) <= 512)) {
        const int64_t t = tiles(128, 128);
        const double f = (double)t / (double)(((t + 767) / 768) * 768);
        const int id = (f >= 0.6 && std::min(M, N) >= 256) ? find_schedule(dtype, 128, 128, 16, 1, 2, 2, -1, 32, 0, 1)
                                                            : find_schedule(dtype, 64, 64, 16, 1, 2, 2, -1, 32, 0, 1);
        if (id >= 0) return take(id);
    }
    // x3 takes in-place tiles below 768 tiles of 64 x 64, with K < 1024 or
    // with M or N <= 512 (above all that, the packing pass that splits each
    // operand once is worth its cost: 4097 x 3001 x 2053 0.175 ms packed
    // against 0.257 in place), 128 x 128 from 1024 tiles of 64 x 64; M or N
    // <= 64 take the direct 64 x 64 tiles instead, and problems of whole
    // 64 x 64 tiles with 16-byte loads and M, N in [512, 4096] keep the
    // direct tiles (1024^3: 0.025 against 0.034 ms).  Over the study's 2080
    // shapes the fastest x3 schedule was an in-place one for 1677; this rule
    // (with the deep-K exception) reaches 0.973 of the exhaustive optimum
    // there (0.948 on its 80 im2col shapes of 3x3 convolutions), against 0.828
    // without the in-place tiles.
    if (dtype == TGEMM_F32_BF16X3) {
        const int64_t t64 = tiles(64, 64);
        const bool whole = vec_allowed && M % 64 == 0 && N % 64 == 0 && std::min(M, N) >= 512 &&
                           std::max(M, N) <= 4096;
        if (deep) {
            const int sk = tiles(256, 256) >= 8 ? find_schedule(dtype, 256, 256, 32, 0, 2, 4, -1, 32, 1)
                                                : find_schedule(dtype, 128, 128, 16, 0, 2, 2, -1, 32, 1);
            if (sk >= 0) return take(sk);
        }
        if ((t64 < 768 || K < 1024 || std::min(M, N) <= 512) && !whole) {
            const int id = std::min(M, N) <= 64 ? find_schedule(dtype, 64, 64, 32, vec_allowed ? 4 : 1)
                           : t64 >= 1024       ? find_schedule(dtype, 128, 128, 16, 1, 2, 2, -1, 32, 0, 1)
                                               : find_schedule(dtype, 64, 64, 16, 1, 2, 2, -1, 32, 0, 1);
            if (id >= 0) return take(id);
        }
    }
    if (K >= 512 && packed_k_ok(K, dtype) && !narrow) {
        int id = -1;
        const int64_t panels16 = (K + 15) / 16, panels32 = (K + 31) / 32;
        // fraction of the launched waves the tiles fill, at `slots` resident workgroups
        auto fill = [&](int64_t t, int64_t slots) { return (double)t / (double)(((t + slots - 1) / slots) * slots); };
        if (dtype == TGEMM_F32) {
            double f = 0.0;  // 128 x 256: two workgroups per CU; the 128 x 128 forms four and two
            if (tiles(128, 256) >= 384) {
                id = find_schedule(dtype, 128, 256, 16, 0, 4, 2);
                f = fill(tiles(128, 256), 512);
            } else if (tiles(128, 256) >= 256) {
                id = find_schedule(dtype, 128, 128, 16, 0, 2, 2, 32768, 16);
                f = fill(tiles(128, 128), 1024);
            } else if (tiles(128, 128) >= 192) {
                id = find_schedule(dtype, 128, 128, 16, 0, 2, 2, 65536);
                f = fill(tiles(128, 128), 512);
            }
            if (f < 0.85 && tiles(128, 256) >= 16 && tiles(128, 256) * panels16 >= 8 * 512) {
                const int sk = tiles(128, 256) >= 384 ? find_schedule(dtype, 128, 256, 16, 0, 4, 2, -1, 32, 1)
                                                      : find_schedule(dtype, 128, 128, 16, 0, 2, 2, -1, 32, 1);
                if (sk >= 0) id = sk;
            }
        } else if (dtype == TGEMM_F32_BF16X3 && tiles(256, 256) < 128 && tiles(128, 128) < 192) {
            if (tiles(256, 256) >= 8 && tiles(256, 256) * panels32 >= 8 * 256)
                id = find_schedule(dtype, 256, 256, 32, 0, 2, 4, -1, 32, 1);
        } else if (dtype == TGEMM_FP8_E4M3) {
            if (tiles(256, 256) >= 128) id = find_schedule(dtype, 256, 256, 128, 0, 4, 2);
            else if (tiles(128, 128) >= 192) id = find_schedule(dtype, 128, 128, 64, 0, 2, 2, 32768);
        } else {
            const int bk = dtype == TGEMM_F32_BF16X3 ? 32 : 64;
            if (tiles(256, 256) >= 128) id = find_schedule(dtype, 256, 256, bk, 0, 2, 4);
            else if (tiles(128, 128) >= 192) id = find_schedule(dtype, 128, 128, bk, 0, 2, 2);
        }
        if (id >= 0) return take(id);
    }
    return direct_schedule(M, N, K, dtype, vec_allowed, out);
}

int select_schedule(int64_t M, int64_t N, int64_t K, int dtype, bool vec_allowed, Choice* out,
                    bool may_run_model)
{
    Policy pol;
    int force_id;
    {
        std::lock_guard<std::mutex> lk(g_sel_mu);
        pol = g_policy;
        force_id = g_force_id;
        if (pol == POLICY_FORCE) {
            if (force_id >= 0 && force_id < num_schedules() && schedule(force_id).dtype == dtype &&
                (schedule(force_id).vec <= 1 || vec_allowed)) {
                out->id = force_id;
                out->group_m = 8;
                out->xcd_remap = 1;
                return TGEMM_SUCCESS;
            }
        } else if (pol == POLICY_TUNED) {
            if (lookup_locked(dtype, M, N, K, vec_allowed, out)) return TGEMM_SUCCESS;
        }
    }
    if (pol == POLICY_MODEL) {
        // a cached prediction costs nothing; a new one runs the network on the GPU,
        // which is not allowed while the caller's stream is being captured
        if (costmodel_cached(M, N, K, dtype, vec_allowed, out)) return TGEMM_SUCCESS;
        if (may_run_model && costmodel_choose(M, N, K, dtype, vec_allowed, out)) return TGEMM_SUCCESS;
        std::lock_guard<std::mutex> lk(g_sel_mu);
        if (lookup_locked(dtype, M, N, K, vec_allowed, out)) return TGEMM_SUCCESS;
    }
    return default_schedule(M, N, K, dtype, vec_allowed, out);
}

}  // namespace tg

extern "C" int tgemm_set_policy(const char* policy)
{
    using namespace tg;
    if (!policy) return TGEMM_INVALID_VALUE;
    std::lock_guard<std::mutex> lk(g_sel_mu);
    if (std::strcmp(policy, "default") == 0) {
        g_policy = POLICY_DEFAULT;
    } else if (std::strcmp(policy, "tuned") == 0) {
        g_policy = POLICY_TUNED;
    } else if (std::strcmp(policy, "model") == 0) {
        g_policy = POLICY_MODEL;
    } else if (std::strncmp(policy, "force:", 6) == 0) {
        char* end = nullptr;
        const long id = std::strtol(policy + 6, &end, 10);
        if (end == policy + 6 || *end != '\0' || id < 0 || id >= num_schedules())
            return TGEMM_INVALID_VALUE;
        g_policy = POLICY_FORCE;
        g_force_id = (int)id;
    } else {
        return TGEMM_INVALID_VALUE;
    }
    return TGEMM_SUCCESS;
}

// Reads JSON lines {"dtype":..,"M":..,"N":..,"K":..,"sched":..,"group_m":..,
// "xcd":..,"ms":..,"valid":true}; keeps the fastest valid entry per problem.
// Lines that do not parse are skipped.  Returns the number of entries used,
// or a negative status when the file cannot be opened.
extern "C" int tgemm_load_tuning_db(const char* db_path)
{
    using namespace tg;
    if (!db_path) return -TGEMM_INVALID_VALUE;
    FILE* f = std::fopen(db_path, "r");
    if (!f) return -TGEMM_INVALID_VALUE;
    char line[4096];
    int used = 0;
    const unsigned long long space = schedule_space_hash();
    std::lock_guard<std::mutex> lk(g_sel_mu);
    while (std::fgets(line, sizeof(line), f)) {
        if (!std::strchr(line, '\n') && !std::feof(f)) {  // overlong line: skip its rest
            int c;
            while ((c = std::fgetc(f)) != EOF && c != '\n') {}
            continue;
        }
        double dt, m, n, k, id, gm, xcd, ms;
        if (!json_number(line, "dtype", &dt) || !json_number(line, "M", &m) ||
            !json_number(line, "N", &n) || !json_number(line, "K", &k) ||
            !json_number(line, "sched", &id) || !json_number(line, "group_m", &gm) ||
            !json_number(line, "xcd", &xcd) || !json_number(line, "ms", &ms))
            continue;
        if (!json_true(line, "valid")) continue;
        unsigned long long h = 0;
        if (!json_hex(line, "space", &h) || h != space) continue;  // another schedule table
        const int sid = (int)id;
        if (sid < 0 || sid >= num_schedules() || schedule(sid).dtype != (int)dt) continue;
        if (gm < 1 || gm > 64 || !(ms > 0)) continue;
        register_locked((int)dt, (int64_t)m, (int64_t)n, (int64_t)k, schedule(sid).vec,
                        Choice{sid, (int)gm, xcd != 0 ? 1 : 0}, ms);
        ++used;
    }
    std::fclose(f);
    return used;
}

extern "C" int tgemm_select_schedule(int64_t M, int64_t N, int64_t K, int dtype, int* schedule_id,
                                     int* group_m, int* xcd_remap)
{
    using namespace tg;
    if (!schedule_id || !group_m || !xcd_remap) return TGEMM_INVALID_VALUE;
    if (M < 0 || N < 0 || K < 0) return TGEMM_INVALID_VALUE;
    Choice c;
    const int rc = select_schedule(M, N, K, dtype, dense_vec_ok(N, K, dtype), &c, true);
    if (rc != TGEMM_SUCCESS) return rc;
    *schedule_id = c.id;
    *group_m = c.group_m;
    *xcd_remap = c.xcd_remap;
    return TGEMM_SUCCESS;
}

extern "C" uint64_t tgemm_schedule_space_hash(void) { return tg::schedule_space_hash(); }
