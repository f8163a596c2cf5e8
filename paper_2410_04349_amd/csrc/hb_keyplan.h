// Per-key-partition plans of libhb (shared by single and batched matching).
#pragma once

#include <cstdint>
#include <utility>
#include <vector>

#include "hb_ctx.h"
#include "hb_internal.h"
#include "hb_plan.h"

namespace hb {

// Resources of one key partition's plans, fixed by the rule set (not by
// the evaluation order), so every order of the same rules reads the same
// gathered feature columns.
struct KeyRes {
    std::vector<uint32_t> int_attr, str_attr, prev;
    std::vector<std::pair<uint32_t, uint32_t>> gram_key;
    std::vector<PredSpec> specs;   // predicates evaluated in this partition, by id
    bool any_ed = false;
    bool any_rule = false;
};

// One key partition ready to match: gathered feature columns, LDS layout
// and the plan (host bytecode, or per-slot plans already on the device).
// One rule's segment of a key plan (emit_code): its first instruction,
// the distinct predicates of its first-stage steps in plan order, and the
// predicate of the guard step it shares with its neighbours (-1: none).
struct RuleSeg {
    uint32_t start = 0;
    std::vector<uint32_t> first_preds;
    int guard_pred = -1;
};

struct KeyPlan {
    std::vector<Instr> code;
    MatchParams mp{};
    DevBuf f64, f32;
    double feat_bytes = 0.0;   // bytes of the feature columns (the match kernel reads each once)
    // learned plans: per-slot plans on the device, the block -> slot map and
    // the choice kernel's counters (read after matching)
    bool own_code = false;
    float predicted[2] = {0.f, 0.f};   // model cost of the listed blocks: heuristic plan, chosen plans
    bool discarded = false;   // the per-block plans were not worth their fetch cost: every block runs slot 0
    bool cost_pending = false;   // choice_cost not yet read back (settle_learned)
    DevBuf dev_code, blk_slot, choice_stats, choice_cost;
};

// Reads back the predicted costs of every learned key plan of `kps` (one
// synchronisation for all) and drops the per-block plans of those whose
// predicted saving is under the context's minimum.  Call once the key plans
// sit where they will stay, before their match parameters are used.
void settle_learned(Ctx* c, std::vector<KeyPlan>& kps);

// The evaluation path of a plan kind (given order or the Section 4.2 plan;
// the learned plan starts from the latter).
std::vector<PathRule> plan_path(const RuleSet& rs, int plan);
bool valid_plan(int plan);   // an hb_plan value

// Builds key `ka`'s partition plan; false if no rule can hold there.
// Learned plans add the blocks kept on the heuristic plan for structural
// reasons to *n_fallback.
bool key_plan(Ctx* c, Relation& rel, RuleSet& rs, int plan, const std::vector<PathRule>& path, size_t ka,
              KeyPlan& kp, bool count, uint64_t* n_fallback);

// Sorts n packed pairs (i << 32) | j (i, j < n_rows) of `pairs` ascending
// into `result` (resized to max(n, 1) entries).
void sort_pairs(Ctx* c, DevBuf& pairs, uint64_t n, uint64_t n_rows, DevBuf& result);

}  // namespace hb
