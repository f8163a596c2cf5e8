/*
 * hboracle -- the CPU oracle for rule-based blocking.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU library, and it is deliberately
 * plain and slow: every function follows a definition from the paper, with
 * no blocking, fusion or reordering beyond what that definition states.
 *
 * What it computes (Section 2, "Rule-based blocking" and Section 4 opening):
 *   Ca(D, Delta) = { (i, j) : some rule phi in Delta has every predicate of
 *                    its precondition X satisfied by the valuation t -> t_i,
 *                    s -> t_j }
 * over the pairs of a partition (Section 2, "Blocking").  With only
 * predicates of the forms t.A = s.A and t.A ~ s.A (a symmetric measure) the
 * two valuations of a pair agree, and each pair is listed once, as i < j.
 * A rule set with a predicate t.A = c or s.A = c, or t.A = s.B or
 * t.A ~ s.B over two different attributes, is "ordered": its valuations of
 * (t_i, t_j) and
 * (t_j, t_i) may differ, and Ca lists every ordered pair (i, j), i != j,
 * whose valuation has a witness.
 * evaluated naively: every rule, every predicate, in input order (the
 * "naive approach" at the start of Section 4).
 *
 * Readings of points the paper leaves open (each also listed in the design
 * notes):
 *   - pairs are reported by 0-based row index, packed as (i << 32) | j
 *     (i the tuple bound to t, j the one bound to s) and sorted ascending;
 *     unordered (i < j) unless the rule set is ordered (above);
 *   - t.A = c holds iff t's A is present and equals c (an int64 constant on
 *     a categorical or int64 attribute); t.A = s.B iff both values are
 *     present and equal (Section 2, "Semantics": tuple relational calculus);
 *     t.A ~ s.B with edit distance iff both strings are present and the
 *     Levenshtein distance from t's A to s's B is at most k; t.A ~ s.B with
 *     q-gram Jaccard iff both strings are present and the Jaccard
 *     similarity of t's A's gram set and s's B's (the same q) is at least
 *     num / den (Section 2, "Predicates": a similarity predicate compares
 *     two attributes of the schema, not necessarily the same one);
 *   - q-gram containment t.A <= s.B, the asymmetric measure of the grammar
 *     (Section 2 allows any similarity, symmetric or asymmetric): both
 *     strings present and |G_q(t.A) & G_q(s.B)| * den >= num * |G_q(t.A)|
 *     (an empty t set is contained in anything); a rule set with it is
 *     ordered even when A = B;
 *   - a missing value fails every predicate, including missing = missing
 *     (Table 1 marks missing values; Example 3 and the Section 4 remark on
 *     (t1, t5) treat a missing value as failing equality and similarity);
 *   - string equality is byte-exact;
 *   - "edit distance" is the Levenshtein distance over bytes (unit-cost
 *     insert, delete, substitute), predicate true iff distance <= k;
 *   - "Jaccard" is q-gram Jaccard similarity over sets of distinct length-q
 *     byte windows, true iff |G_a & G_b| / |G_a | G_b| >= num/den, tested as
 *     |I| * den >= num * |U| in integers; a non-empty string shorter than q
 *     has the gram set {s}; the empty string has the empty set; two empty
 *     sets have similarity 1;
 *   - the numeric range predicate is |a - b| <= d over int64, in 128 bits;
 *   - blocked mode: each rule's blocking key is its first equality predicate
 *     on a categorical or int64 attribute (input order); candidate pairs are
 *     the pairs sharing a key value under some rule's key (partitions of
 *     Section 2, "Data partitioning"); since that equality is one of the
 *     rule's own predicates, blocked mode equals full mode.
 */
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <vector>

extern "C" {

enum { ORA_STRING = 0, ORA_CATEGORICAL = 1, ORA_INT64 = 2 };
enum { ORA_EQ = 0, ORA_ED = 1, ORA_JACCARD = 2, ORA_ABSDIFF = 3, ORA_CONST = 4, ORA_CROSS = 5, ORA_ED_CROSS = 6,
       ORA_JACCARD_CROSS = 7, ORA_CONTAIN = 8 };

struct ora_col {
    int32_t type;
    const uint64_t* offsets;
    const uint8_t* data;
    const int64_t* values;
    const uint8_t* valid;
};

struct ora_pred {
    int32_t op;
    uint32_t attr;
    int64_t k;
    uint32_t q;
    uint32_t num;
    uint32_t den;
    int64_t d;
    uint32_t attr_b;  /* ORA_CROSS, ORA_ED_CROSS, ORA_JACCARD_CROSS, ORA_CONTAIN: the attribute B of t.A = s.B,
                         t.A ~ s.B */
    int32_t side;     /* ORA_CONST: 0 for t.A = c, 1 for s.A = c */
    int64_t c;        /* ORA_CONST: the constant */
};

}  // extern "C"

namespace {

bool is_valid(const ora_col& c, uint64_t i) {
    if (!c.valid) return true;
    return (c.valid[i >> 3] >> (i & 7)) & 1;
}

std::string str_at(const ora_col& c, uint64_t i) {
    return std::string(reinterpret_cast<const char*>(c.data + c.offsets[i]),
                       reinterpret_cast<const char*>(c.data + c.offsets[i + 1]));
}

/* Levenshtein distance by the full Wagner-Fischer table:
 * D[x][0] = x, D[0][y] = y,
 * D[x][y] = min(D[x-1][y] + 1, D[x][y-1] + 1, D[x-1][y-1] + [a_x != b_y]). */
int64_t levenshtein(const std::string& a, const std::string& b) {
    const size_t m = a.size(), n = b.size();
    std::vector<std::vector<int64_t>> D(m + 1, std::vector<int64_t>(n + 1, 0));
    for (size_t x = 0; x <= m; ++x) D[x][0] = (int64_t)x;
    for (size_t y = 0; y <= n; ++y) D[0][y] = (int64_t)y;
    for (size_t x = 1; x <= m; ++x)
        for (size_t y = 1; y <= n; ++y) {
            int64_t sub = D[x - 1][y - 1] + (a[x - 1] != b[y - 1] ? 1 : 0);
            int64_t del = D[x - 1][y] + 1;
            int64_t ins = D[x][y - 1] + 1;
            D[x][y] = std::min(sub, std::min(del, ins));
        }
    return D[m][n];
}

/* G_q(s): distinct length-q windows; {s} if 0 < |s| < q; empty if |s| = 0 */
std::set<std::string> qgrams(const std::string& s, uint32_t q) {
    std::set<std::string> g;
    if (s.empty()) return g;
    if (s.size() < q) { g.insert(s); return g; }
    for (size_t x = 0; x + q <= s.size(); ++x) g.insert(s.substr(x, q));
    return g;
}

void inter_union(const std::set<std::string>& A, const std::set<std::string>& B,
                 uint64_t* I, uint64_t* U) {
    std::set<std::string> inter, uni;
    std::set_intersection(A.begin(), A.end(), B.begin(), B.end(), std::inserter(inter, inter.begin()));
    std::set_union(A.begin(), A.end(), B.begin(), B.end(), std::inserter(uni, uni.begin()));
    *I = inter.size();
    *U = uni.size();
}

bool jaccard_ge(uint64_t I, uint64_t U, uint32_t num, uint32_t den) {
    if (U == 0) return true; /* J(empty, empty) = 1 */
    return (unsigned __int128)I * den >= (unsigned __int128)num * U;
}

/* Per-(attribute, q) cache of gram sets: each tuple's set G_q(s) is a
 * function of the tuple alone, so it is built once per tuple. */
struct GramCache {
    std::map<std::pair<uint32_t, uint32_t>, std::vector<std::set<std::string>>> sets;
    void add(const ora_col* cols, uint64_t n, uint32_t attr, uint32_t q) {
        auto key = std::make_pair(attr, q);
        if (sets.count(key)) return;
        const ora_col& c = cols[attr];
        std::vector<std::set<std::string>> v(n);
        for (uint64_t i = 0; i < n; ++i)
            if (is_valid(c, i)) v[i] = qgrams(str_at(c, i), q);
        sets.emplace(key, std::move(v));
    }
    void build(const ora_col* cols, uint64_t n, const ora_pred* preds, size_t np) {
        for (size_t p = 0; p < np; ++p) {
            if (preds[p].op == ORA_JACCARD) add(cols, n, preds[p].attr, preds[p].q);
            if (preds[p].op == ORA_JACCARD_CROSS || preds[p].op == ORA_CONTAIN) {
                add(cols, n, preds[p].attr, preds[p].q);
                add(cols, n, preds[p].attr_b, preds[p].q);
            }
        }
    }
};

/* h(t_i, t_j) |= p, with h(t) = t_i and h(s) = t_j */
bool sat(const ora_col* cols, const ora_pred& p, uint64_t i, uint64_t j, const GramCache* gc) {
    const ora_col& c = cols[p.attr];
    if (p.op == ORA_CONST) {
        const uint64_t row = p.side == 0 ? i : j;
        return is_valid(c, row) && c.values[row] == p.c;
    }
    if (p.op == ORA_CROSS) {
        const ora_col& b = cols[p.attr_b];
        return is_valid(c, i) && is_valid(b, j) && c.values[i] == b.values[j];
    }
    if (p.op == ORA_ED_CROSS) {
        const ora_col& b = cols[p.attr_b];
        return is_valid(c, i) && is_valid(b, j) && levenshtein(str_at(c, i), str_at(b, j)) <= p.k;
    }
    if (p.op == ORA_JACCARD_CROSS) {   /* J(G_q(t.A), G_q(s.B)) >= num / den */
        const ora_col& b = cols[p.attr_b];
        if (!is_valid(c, i) || !is_valid(b, j)) return false;
        uint64_t I, U;
        if (gc) {
            inter_union(gc->sets.at(std::make_pair(p.attr, p.q))[i], gc->sets.at(std::make_pair(p.attr_b, p.q))[j],
                        &I, &U);
        } else {
            inter_union(qgrams(str_at(c, i), p.q), qgrams(str_at(b, j), p.q), &I, &U);
        }
        return jaccard_ge(I, U, p.num, p.den);
    }
    if (p.op == ORA_CONTAIN) {   /* |G_q(t.A) & G_q(s.B)| / |G_q(t.A)| >= num / den */
        const ora_col& b = cols[p.attr_b];
        if (!is_valid(c, i) || !is_valid(b, j)) return false;
        uint64_t I, U;
        uint64_t nt;
        if (gc) {
            const auto& ga = gc->sets.at(std::make_pair(p.attr, p.q))[i];
            inter_union(ga, gc->sets.at(std::make_pair(p.attr_b, p.q))[j], &I, &U);
            nt = ga.size();
        } else {
            const std::set<std::string> ga = qgrams(str_at(c, i), p.q);
            inter_union(ga, qgrams(str_at(b, j), p.q), &I, &U);
            nt = ga.size();
        }
        (void)U;
        return (unsigned __int128)I * p.den >= (unsigned __int128)p.num * nt;
    }
    if (!is_valid(c, i) || !is_valid(c, j)) return false;
    switch (p.op) {
    case ORA_EQ:
        if (c.type == ORA_STRING) return str_at(c, i) == str_at(c, j);
        return c.values[i] == c.values[j];
    case ORA_ABSDIFF: {
        __int128 diff = (__int128)c.values[i] - (__int128)c.values[j];
        if (diff < 0) diff = -diff;
        return diff <= (__int128)p.d;
    }
    case ORA_ED:
        return levenshtein(str_at(c, i), str_at(c, j)) <= p.k;
    case ORA_JACCARD: {
        uint64_t I, U;
        if (gc) {
            const auto& v = gc->sets.at(std::make_pair(p.attr, p.q));
            inter_union(v[i], v[j], &I, &U);
        } else {
            inter_union(qgrams(str_at(c, i), p.q), qgrams(str_at(c, j), p.q), &I, &U);
        }
        return jaccard_ge(I, U, p.num, p.den);
    }
    }
    return false;
}

struct RuleSet {
    std::vector<std::vector<ora_pred>> rules;
};

/* Does some predicate tell t from s (a constant on one side, or a
 * comparison across two different attributes)? */
bool ordered_rules(const RuleSet& rs) {
    for (const auto& rule : rs.rules)
        for (const auto& p : rule)
            if (p.op == ORA_CONST || p.op == ORA_CONTAIN ||
                ((p.op == ORA_CROSS || p.op == ORA_ED_CROSS || p.op == ORA_JACCARD_CROSS) && p.attr != p.attr_b))
                return true;
    return false;
}

RuleSet unpack_rules(uint32_t n_rules, const uint32_t* rule_len, const ora_pred* preds) {
    RuleSet rs;
    size_t off = 0;
    for (uint32_t r = 0; r < n_rules; ++r) {
        rs.rules.emplace_back(preds + off, preds + off + rule_len[r]);
        off += rule_len[r];
    }
    return rs;
}

/* (t_i, t_j) in Ca iff some rule is a witness: every predicate holds */
bool witness_exists(const ora_col* cols, const RuleSet& rs, uint64_t i, uint64_t j, const GramCache* gc) {
    for (const auto& rule : rs.rules) {
        bool all = true;
        for (const auto& p : rule)
            if (!sat(cols, p, i, j, gc)) { all = false; break; }
        if (all) return true;
    }
    return false;
}

/* first equality on a categorical / int64 attribute, in input order; -1 if none */
int64_t rule_key(const ora_col* cols, const std::vector<ora_pred>& rule) {
    for (const auto& p : rule)
        if (p.op == ORA_EQ && (cols[p.attr].type == ORA_CATEGORICAL || cols[p.attr].type == ORA_INT64))
            return p.attr;
    return -1;
}

std::vector<uint32_t> distinct_keys(const ora_col* cols, const RuleSet& rs, bool* ok) {
    std::vector<uint32_t> keys;
    *ok = true;
    for (const auto& rule : rs.rules) {
        int64_t k = rule_key(cols, rule);
        if (k < 0) { *ok = false; continue; }
        if (std::find(keys.begin(), keys.end(), (uint32_t)k) == keys.end()) keys.push_back((uint32_t)k);
    }
    return keys;
}

/* groups of rows sharing a value of each key attribute (missing keys join no group) */
std::vector<std::vector<uint64_t>> key_groups(const ora_col* cols, const std::vector<uint32_t>& keys, uint64_t n) {
    std::vector<std::vector<uint64_t>> groups;
    for (uint32_t k : keys) {
        std::map<int64_t, std::vector<uint64_t>> g;
        for (uint64_t i = 0; i < n; ++i)
            if (is_valid(cols[k], i)) g[cols[k].values[i]].push_back(i);
        for (auto& kv : g)
            if (kv.second.size() >= 2) groups.push_back(std::move(kv.second));
    }
    return groups;
}

uint64_t pack(uint64_t i, uint64_t j) { return (std::min(i, j) << 32) | std::max(i, j); }

}  // namespace

extern "C" {

int64_t ora_levenshtein(const uint8_t* a, uint64_t la, const uint8_t* b, uint64_t lb) {
    return levenshtein(std::string((const char*)a, la), std::string((const char*)b, lb));
}

/* |G_q(a)|, |G_q(a) & G_q(b)|, |G_q(a) | G_q(b)| */
void ora_qgram_stats(const uint8_t* a, uint64_t la, const uint8_t* b, uint64_t lb, uint32_t q,
                     uint64_t* size_a, uint64_t* inter, uint64_t* uni) {
    auto A = qgrams(std::string((const char*)a, la), q);
    auto B = qgrams(std::string((const char*)b, lb), q);
    *size_a = A.size();
    inter_union(A, B, inter, uni);
}

int ora_ordered(uint32_t n_rules, const uint32_t* rule_len, const ora_pred* preds) {
    return ordered_rules(unpack_rules(n_rules, rule_len, preds)) ? 1 : 0;
}

int ora_jaccard_ge(const uint8_t* a, uint64_t la, const uint8_t* b, uint64_t lb, uint32_t q,
                   uint32_t num, uint32_t den) {
    uint64_t I, U;
    inter_union(qgrams(std::string((const char*)a, la), q), qgrams(std::string((const char*)b, lb), q), &I, &U);
    return jaccard_ge(I, U, num, den) ? 1 : 0;
}

int ora_sat(const ora_col* cols, const ora_pred* p, uint64_t i, uint64_t j) {
    return sat(cols, *p, i, j, nullptr) ? 1 : 0;
}

/* Is rule r (given as n_preds predicates) a witness at (i, j)? */
int ora_rule_witness(const ora_col* cols, uint32_t n_preds, const ora_pred* preds, uint64_t i, uint64_t j) {
    for (uint32_t p = 0; p < n_preds; ++p)
        if (!sat(cols, preds[p], i, j, nullptr)) return 0;
    return 1;
}

/* Ca(D, Delta) as a sorted list of packed pairs.
 * mode 0: blocked (pairs sharing some rule's key); mode 1: every pair of
 * rows (both orders for an ordered rule set).
 * Returns the number of pairs (written up to `cap`), -2 if a rule has no
 * key in blocked mode. */
int64_t ora_blocking(const ora_col* cols, uint32_t n_cols, uint64_t n_rows, uint32_t n_rules,
                     const uint32_t* rule_len, const ora_pred* preds, int mode, int n_threads,
                     uint64_t* out, uint64_t cap) {
    (void)n_cols;
    RuleSet rs = unpack_rules(n_rules, rule_len, preds);
    size_t np = 0;
    for (uint32_t r = 0; r < n_rules; ++r) np += rule_len[r];
    GramCache gc;
    gc.build(cols, n_rows, preds, np);
    if (n_threads < 1) n_threads = 1;
    const bool ordered = ordered_rules(rs);

    std::vector<uint64_t> result;
    std::mutex mu;
    if (mode == 1) {
        std::atomic<uint64_t> next{0};
        auto work = [&]() {
            std::vector<uint64_t> local;
            for (;;) {
                uint64_t i = next.fetch_add(1);
                if (i >= n_rows) break;
                for (uint64_t j = i + 1; j < n_rows; ++j) {
                    if (!ordered) {
                        if (witness_exists(cols, rs, i, j, &gc)) local.push_back(pack(i, j));
                        continue;
                    }
                    if (witness_exists(cols, rs, i, j, &gc)) local.push_back((i << 32) | j);
                    if (witness_exists(cols, rs, j, i, &gc)) local.push_back((j << 32) | i);
                }
            }
            std::lock_guard<std::mutex> g(mu);
            result.insert(result.end(), local.begin(), local.end());
        };
        std::vector<std::thread> th;
        for (int t = 0; t < n_threads; ++t) th.emplace_back(work);
        for (auto& t : th) t.join();
    } else {
        bool ok;
        std::vector<uint32_t> keys = distinct_keys(cols, rs, &ok);
        if (!ok) return -2;
        auto groups = key_groups(cols, keys, n_rows);
        std::sort(groups.begin(), groups.end(),
                  [](const std::vector<uint64_t>& a, const std::vector<uint64_t>& b) { return a.size() > b.size(); });
        std::atomic<size_t> next{0};
        auto work = [&]() {
            std::vector<uint64_t> local;
            for (;;) {
                size_t g = next.fetch_add(1);
                if (g >= groups.size()) break;
                const auto& rows = groups[g];
                for (size_t x = 0; x < rows.size(); ++x)
                    for (size_t y = x + 1; y < rows.size(); ++y) {
                        const uint64_t a = rows[x], b = rows[y];
                        if (!ordered) {
                            if (witness_exists(cols, rs, a, b, &gc)) local.push_back(pack(a, b));
                            continue;
                        }
                        if (witness_exists(cols, rs, a, b, &gc)) local.push_back((a << 32) | b);
                        if (witness_exists(cols, rs, b, a, &gc)) local.push_back((b << 32) | a);
                    }
            }
            std::lock_guard<std::mutex> g(mu);
            result.insert(result.end(), local.begin(), local.end());
        };
        std::vector<std::thread> th;
        for (int t = 0; t < n_threads; ++t) th.emplace_back(work);
        for (auto& t : th) t.join();
    }
    std::sort(result.begin(), result.end());
    result.erase(std::unique(result.begin(), result.end()), result.end());
    for (uint64_t x = 0; x < result.size() && x < cap; ++x) out[x] = result[x];
    return (int64_t)result.size();
}

/* Number of distinct pairs i < j that share a value of some rule's key,
 * by enumeration.  -2 if a rule has no key. */
int64_t ora_candidate_count(const ora_col* cols, uint64_t n_rows, uint32_t n_rules,
                            const uint32_t* rule_len, const ora_pred* preds) {
    RuleSet rs = unpack_rules(n_rules, rule_len, preds);
    bool ok;
    std::vector<uint32_t> keys = distinct_keys(cols, rs, &ok);
    if (!ok) return -2;
    auto groups = key_groups(cols, keys, n_rows);
    std::vector<uint64_t> all;
    for (const auto& rows : groups)
        for (size_t x = 0; x < rows.size(); ++x)
            for (size_t y = x + 1; y < rows.size(); ++y) all.push_back(pack(rows[x], rows[y]));
    std::sort(all.begin(), all.end());
    all.erase(std::unique(all.begin(), all.end()), all.end());
    return (int64_t)all.size();
}

/* For each given pair (packed (i << 32) | j), flags[x] = 1 iff some rule
 * is a witness at the valuation t -> t_i, s -> t_j, by the definition (no
 * blocking involved). */
int ora_eval_pairs(const ora_col* cols, uint64_t n_rows, uint32_t n_rules, const uint32_t* rule_len,
                   const ora_pred* preds, const uint64_t* pairs, uint64_t n_pairs, int n_threads,
                   uint8_t* flags) {
    RuleSet rs = unpack_rules(n_rules, rule_len, preds);
    size_t np = 0;
    for (uint32_t r = 0; r < n_rules; ++r) np += rule_len[r];
    GramCache gc;
    gc.build(cols, n_rows, preds, np);
    if (n_threads < 1) n_threads = 1;
    std::atomic<uint64_t> next{0};
    const uint64_t chunk = 4096;
    auto work = [&]() {
        for (;;) {
            uint64_t s = next.fetch_add(chunk);
            if (s >= n_pairs) break;
            uint64_t e = std::min(n_pairs, s + chunk);
            for (uint64_t x = s; x < e; ++x) {
                uint64_t i = pairs[x] >> 32, j = pairs[x] & 0xFFFFFFFFull;
                flags[x] = (i != j && witness_exists(cols, rs, i, j, &gc)) ? 1 : 0;
            }
        }
    };
    std::vector<std::thread> th;
    for (int t = 0; t < n_threads; ++t) th.emplace_back(work);
    for (auto& t : th) t.join();
    return 0;
}

}  // extern "C"
