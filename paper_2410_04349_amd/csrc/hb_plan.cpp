// Host-side execution-plan generator of libhb (Section 4.2), pure C++.
//
// Input: per distinct predicate an estimated selectivity sp (probability of
// being satisfied) and a normalised cost; rules as lists of predicate ids.
// The ranking of step 1 can be swapped for cheapest-first or most-selective-
// first, and the resulting path's predicate or rule order shuffled: the
// ordering strategies the paper's experiments compare EPG with.
//
// Output: the sequential execution path of Section 5.1 -- rules in the
// order a depth-first walk of the execution tree reaches their leaves, each
// with its predicates in root-to-leaf order.
//
//  1. order predicates by (1 - sp) / cost, largest first (ties: smaller id);
//  2. insert every rule, its predicates sorted by that order, into a prefix
//     tree, re-using a child edge that carries the same predicate;
//  3. a rule's witness probability is the product of its predicates' sp,
//     and an edge's score is the largest witness probability among the rules
//     whose root-to-leaf path contains the edge;
//  4. walk the tree depth first, children by decreasing score (ties: the
//     order the edges were created).  A rule ending at a node is listed on
//     arrival there, before the node's children, since reaching the node
//     already makes it a witness.
#include "hb_plan.h"

#include <algorithm>
#include <functional>

namespace hb {

namespace {

struct TreeNode {
    int pred = -1;
    std::vector<int> children;   // node ids in creation order
    std::vector<uint32_t> ends;  // rules whose path ends here
    double score = 0.0;
};

}  // namespace

std::vector<PathRule> given_path(const std::vector<std::vector<uint32_t>>& rules) {
    std::vector<PathRule> out;
    for (uint32_t r = 0; r < rules.size(); ++r) {
        PathRule pr;
        pr.rule = r;
        for (uint32_t p : rules[r])
            if (std::find(pr.preds.begin(), pr.preds.end(), p) == pr.preds.end()) pr.preds.push_back(p);
        out.push_back(pr);
    }
    return out;
}

std::vector<PathRule> epg_path(const std::vector<double>& sp, const std::vector<double>& cost,
                               const std::vector<std::vector<uint32_t>>& rules, Rank by) {
    const size_t np = sp.size();
    std::vector<double> ce(np);   // larger ranks first
    for (size_t p = 0; p < np; ++p)
        ce[p] = by == Rank::kCheapest ? -cost[p] : by == Rank::kMostSelective ? 1.0 - sp[p]
                                                                              : (1.0 - sp[p]) / cost[p];
    std::vector<uint32_t> order(np);
    for (size_t p = 0; p < np; ++p) order[p] = (uint32_t)p;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return ce[a] > ce[b]; });
    std::vector<size_t> rank(np);
    for (size_t x = 0; x < np; ++x) rank[order[x]] = x;

    std::vector<TreeNode> nodes(1);
    std::vector<std::vector<int>> paths(rules.size());
    for (uint32_t r = 0; r < rules.size(); ++r) {
        std::vector<uint32_t> ps;
        for (uint32_t p : rules[r])
            if (std::find(ps.begin(), ps.end(), p) == ps.end()) ps.push_back(p);
        std::sort(ps.begin(), ps.end(), [&](uint32_t a, uint32_t b) { return rank[a] < rank[b]; });
        int node = 0;
        for (uint32_t p : ps) {
            int next = -1;
            for (int c : nodes[node].children)
                if (nodes[c].pred == (int)p) { next = c; break; }
            if (next < 0) {
                next = (int)nodes.size();
                TreeNode nn;
                nn.pred = (int)p;
                nodes.push_back(nn);
                nodes[node].children.push_back(next);
            }
            node = next;
            paths[r].push_back(node);
        }
        nodes[node].ends.push_back(r);
    }

    // witness probability, with the product taken over predicate ids in
    // ascending order so that equal inputs give identical doubles
    for (uint32_t r = 0; r < rules.size(); ++r) {
        std::vector<uint32_t> ids(rules[r].begin(), rules[r].end());
        std::sort(ids.begin(), ids.end());
        ids.erase(std::unique(ids.begin(), ids.end()), ids.end());
        double wp = 1.0;
        for (uint32_t p : ids) wp *= sp[p];
        for (int nd : paths[r]) nodes[nd].score = std::max(nodes[nd].score, wp);
    }

    std::vector<PathRule> out;
    std::function<void(int)> visit = [&](int nd) {
        std::vector<uint32_t> ends = nodes[nd].ends;
        std::sort(ends.begin(), ends.end());
        for (uint32_t r : ends) {
            PathRule pr;
            pr.rule = r;
            for (int x : paths[r]) pr.preds.push_back((uint32_t)nodes[x].pred);
            out.push_back(pr);
        }
        std::vector<int> kids = nodes[nd].children;
        std::stable_sort(kids.begin(), kids.end(), [&](int a, int b) { return nodes[a].score > nodes[b].score; });
        for (int c : kids) visit(c);
    };
    visit(0);
    return out;
}

std::vector<PathRule> shuffled_path(std::vector<PathRule> path, bool shuffle_preds, bool shuffle_rules,
                                    uint64_t seed) {
    uint64_t st = seed;
    auto next = [&st]() {   // splitmix64 (Steele, Lea and Flood)
        uint64_t z = (st += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    auto shuffle = [&next](auto& v) {   // Fisher-Yates
        for (size_t i = v.size(); i > 1; --i) std::swap(v[i - 1], v[next() % i]);
    };
    if (shuffle_preds)
        for (PathRule& pr : path) shuffle(pr.preds);
    if (shuffle_rules) shuffle(path);
    return path;
}

}  // namespace hb
