// Schedule selection (Tiramisu paper, Section VI-A: tile sizes are chosen by
// measurement on the target machine).  Policies: a built-in rule, the tuning
// database written by the autotuner, or one forced schedule.
#pragma once
#include <stdint.h>

namespace tg {

struct Choice {
    int id;
    int group_m;
    int xcd_remap;
};

// Picks a schedule for the current policy; vec_allowed says whether the
// operands permit 16-byte loads; may_run_model is false while the caller's
// stream is being captured (a new cost-model prediction runs GPU work).
int select_schedule(int64_t M, int64_t N, int64_t K, int dtype, bool vec_allowed, Choice* out,
                    bool may_run_model = true);

// Cost-model answers for the "model" policy (false: no model, out of range).
bool costmodel_choose(int64_t M, int64_t N, int64_t K, int dtype, bool vec_allowed, Choice* out);
bool costmodel_cached(int64_t M, int64_t N, int64_t K, int dtype, bool vec_allowed, Choice* out);

// Built-in rule only (also the fallback of the other policies).
int default_schedule(int64_t M, int64_t N, int64_t K, int dtype, bool vec_allowed, Choice* out);

// Built-in rule restricted to schedules that need no workspace.
int direct_schedule(int64_t M, int64_t N, int64_t K, int dtype, bool vec_allowed, Choice* out);

// Index of the compiled schedule with these parameters, or -1 (split: 1 for
// the stream-K form of a packed schedule; inplace: 1 for an in-place one).
int find_schedule(int dtype, int BM, int BN, int BK, int vec, int WGM = 2, int WGN = 2, int lds = -1,
                  int mfma = 32, int split = 0, int inplace = 0);

// Tuned choices (filled by the autotuner and by the database loader).
void register_tuned(int dtype, int64_t M, int64_t N, int64_t K, int vec, const Choice& c, double ms);
bool lookup_tuned(int dtype, int64_t M, int64_t N, int64_t K, int vec, Choice* out);

// Whether 16-byte loads are possible for a dense problem (row strides K and N)
// whose base pointers are 16-byte aligned: the case the autotuner measures.
bool dense_vec_ok(int64_t N, int64_t K, int dtype);

// Hash of the compiled schedule table; tuning records of another table are ignored.
uint64_t schedule_space_hash();

}  // namespace tg
