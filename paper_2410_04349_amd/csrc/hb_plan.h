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

// The sequential execution path of the execution tree built from the
// estimates (Section 4.2 ordering, tree, edge scores, DFS order).
std::vector<PathRule> epg_path(const std::vector<double>& sp, const std::vector<double>& cost,
                               const std::vector<std::vector<uint32_t>>& rules);

}  // namespace hb
