// Host-side execution-plan generator of libhb (Section 4.2).
#pragma once

#include <cstdint>
#include <vector>

namespace hb {

struct PathRule {
    uint32_t rule;
    std::vector<uint32_t> preds;    // distinct predicate ids in evaluation order
    std::vector<uint32_t> verify;   // order of the exact checks (empty: as `preds`)
};

// Rules and predicates in the given order (duplicates within a rule dropped).
std::vector<PathRule> given_path(const std::vector<std::vector<uint32_t>>& rules);

// Predicate ranking of the execution tree: the paper's cost-effectiveness
// (1 - sp) / cost, or one of the single-criterion orders its experiments
// compare against (cheapest first; most selective, i.e. lowest sp, first).
enum class Rank { kCostEffective, kCheapest, kMostSelective };

// The sequential execution path of the execution tree built from the
// estimates (Section 4.2 ordering, tree, edge scores, DFS order), with the
// predicates ranked by `rank`.
std::vector<PathRule> epg_path(const std::vector<double>& sp, const std::vector<double>& cost,
                               const std::vector<std::vector<uint32_t>>& rules,
                               Rank rank = Rank::kCostEffective);

// The heuristic path with each rule's predicates (shuffle_preds) or the
// rule order (shuffle_rules) permuted at random from `seed` (the
// experiments' random-order variants).
std::vector<PathRule> shuffled_path(std::vector<PathRule> path, bool shuffle_preds, bool shuffle_rules,
                                    uint64_t seed);

}  // namespace hb
