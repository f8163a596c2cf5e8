// C-ABI entry points of libhb: context, relation load, rule compilation,
// key partitioning and pair matching.  Host orchestration only; every step
// on the data runs in this library's HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/hb.h"
#include "hb_ctx.h"
#include "hb_internal.h"
#include "hb_abi.h"
#include "hb_keyplan.h"
#include "hb_plan.h"

namespace hb {

// ------------------------------------------------------------ load

// Asynchronous load: every copy and the offset validation run on the
// context's copy stream; the relation is finished (its validation read
// back, its column table uploaded) when a later call first uses it.
static void load_relation_async(Ctx* c, uint32_t n_rows, uint32_t n_cols, const hb_column* cols, int on_device,
                                uint32_t* rel_id) {
    if (!cols || !rel_id) fail(HB_ERR_INVALID_ARG, "NULL argument");
    if (n_rows == 0 || n_rows >= 0x80000000u) fail(HB_ERR_INVALID_ARG, "n_rows must be in [1, 2^31)");
    if (n_cols == 0 || n_cols > 256) fail(HB_ERR_INVALID_ARG, "n_cols must be in [1, 256]");
    if (!c->copy_stream) HB_HIP(hipStreamCreateWithFlags(&c->copy_stream, hipStreamNonBlocking));
    hipStream_t cs = c->copy_stream;
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    auto rel = std::make_unique<Relation>();
    rel->n_rows = n_rows;
    rel->n_cols = n_cols;
    rel->cols.resize(n_cols);
    const size_t vbytes = (n_rows + 7) / 8;
    // allocations are stream-ordered on the context stream; the copy stream
    // starts after them
    rel->load_stats.alloc(c, 32 * (size_t)n_cols);
    zero(c, rel->load_stats.get(), rel->load_stats.size());
    for (uint32_t a = 0; a < n_cols; ++a) {
        const hb_column& in = cols[a];
        Column& col = rel->cols[a];
        col.type = in.type;
        if (in.type == HB_COL_STRING) {
            if (!in.offsets) fail(HB_ERR_INVALID_ARG, "string column " + std::to_string(a) + " has no offsets");
            if (!in.bytes) fail(HB_ERR_INVALID_ARG, "string column " + std::to_string(a) + " has no bytes");
            col.off.alloc(c, sizeof(uint64_t) * ((size_t)n_rows + 1));
        } else if (in.type == HB_COL_CATEGORICAL || in.type == HB_COL_INT64) {
            if (!in.values) fail(HB_ERR_INVALID_ARG, "column " + std::to_string(a) + " has no values");
            col.values.alloc(c, sizeof(int64_t) * n_rows);
        } else {
            fail(HB_ERR_INVALID_ARG, "column " + std::to_string(a) + " has an unknown type");
        }
        if (in.valid) col.valid.alloc(c, vbytes);
    }
    hipEvent_t allocated;
    HB_HIP(hipEventCreateWithFlags(&allocated, hipEventDisableTiming));
    HB_HIP(hipEventRecord(allocated, c->stream));
    HB_HIP(hipStreamWaitEvent(cs, allocated, 0));
    (void)hipEventDestroy(allocated);
    for (uint32_t a = 0; a < n_cols; ++a) {
        const hb_column& in = cols[a];
        Column& col = rel->cols[a];
        if (in.type == HB_COL_STRING) {
            HB_HIP(hipMemcpyAsync(col.off.get(), in.offsets, sizeof(uint64_t) * ((size_t)n_rows + 1), kind, cs));
            uint8_t* st = rel->load_stats.as<uint8_t>() + 32 * a;
            HB_HIP(launch_string_stats(col.off.as<uint64_t>(), n_rows, (uint32_t*)st, (unsigned long long*)(st + 8),
                                       (uint32_t*)(st + 16), cs));
        } else if (in.type == HB_COL_CATEGORICAL || in.type == HB_COL_INT64) {
            HB_HIP(hipMemcpyAsync(col.values.get(), in.values, sizeof(int64_t) * n_rows, kind, cs));
        }
        if (in.valid) HB_HIP(hipMemcpyAsync(col.valid.get(), in.valid, vbytes, kind, cs));
    }
    // the byte arenas: their sizes are the offsets' last entries
    for (uint32_t a = 0; a < n_cols; ++a) {
        const hb_column& in = cols[a];
        if (in.type != HB_COL_STRING) continue;
        Column& col = rel->cols[a];
        uint64_t total;
        if (on_device) {
            HB_HIP(hipMemcpyAsync(&total, in.offsets + n_rows, 8, hipMemcpyDeviceToHost, cs));
            HB_HIP(hipStreamSynchronize(cs));
        } else {
            total = in.offsets[n_rows];
        }
        col.bytes.alloc(c, total + 16);
        hipEvent_t e;
        HB_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        HB_HIP(hipEventRecord(e, c->stream));
        HB_HIP(hipStreamWaitEvent(cs, e, 0));
        (void)hipEventDestroy(e);
        if (total) HB_HIP(hipMemcpyAsync(col.bytes.get(), in.bytes, total, kind, cs));
    }
    HB_HIP(hipEventCreateWithFlags(&rel->ready, hipEventDisableTiming));
    HB_HIP(hipEventRecord(rel->ready, cs));
    rel->pending = true;
    rel->id = c->next_id++;
    *rel_id = rel->id;
    c->rels[rel->id] = std::move(rel);
}

void finish_load(Ctx* c, Relation& rel) {
    HB_HIP(hipStreamWaitEvent(c->stream, rel.ready, 0));
    std::vector<uint32_t> h(8 * (size_t)rel.n_cols);
    HB_HIP(hipMemcpyAsync(h.data(), rel.load_stats.get(), 32 * (size_t)rel.n_cols, hipMemcpyDeviceToHost, c->stream));
    c->sync();
    // invalid offsets keep the relation unusable (every use reports them);
    // it can still be released
    for (uint32_t a = 0; a < rel.n_cols; ++a)
        if (rel.cols[a].type == HB_COL_STRING && h[8 * (size_t)a + 4])
            fail(HB_ERR_INVALID_ARG, "string offsets of column " + std::to_string(a) + " are invalid");
    (void)hipEventDestroy(rel.ready);
    rel.ready = nullptr;
    rel.pending = false;
    rel.h_cols.resize(rel.n_cols);
    for (uint32_t a = 0; a < rel.n_cols; ++a) {
        Column& col = rel.cols[a];
        if (col.type == HB_COL_STRING) {
            const uint32_t* st = h.data() + 8 * (size_t)a;
            col.max_len = st[0];
            uint64_t tot;
            std::memcpy(&tot, st + 2, 8);
            col.mean_len = (double)tot / (double)rel.n_rows;
        }
        ColDev d{};
        d.type = col.type;
        d.max_len = col.max_len;
        d.off = col.off.as<uint64_t>();
        d.bytes = col.bytes.as<uint8_t>();
        d.values = col.values.as<int64_t>();
        d.valid = col.valid.as<uint8_t>();
        rel.h_cols[a] = d;
    }
    rel.d_cols.alloc(c, sizeof(ColDev) * rel.n_cols);
    HB_HIP(hipMemcpyAsync(rel.d_cols.get(), rel.h_cols.data(), sizeof(ColDev) * rel.n_cols, hipMemcpyHostToDevice,
                          c->stream));
    rel.load_stats.release();
}

static void load_relation(Ctx* c, uint32_t n_rows, uint32_t n_cols, const hb_column* cols, int on_device,
                          uint32_t* rel_id) {
    if (!cols || !rel_id) fail(HB_ERR_INVALID_ARG, "NULL argument");
    if (n_rows == 0 || n_rows >= 0x80000000u) fail(HB_ERR_INVALID_ARG, "n_rows must be in [1, 2^31)");
    if (n_cols == 0 || n_cols > 256) fail(HB_ERR_INVALID_ARG, "n_cols must be in [1, 256]");
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    auto rel = std::make_unique<Relation>();
    rel->n_rows = n_rows;
    rel->n_cols = n_cols;
    rel->cols.resize(n_cols);
    const size_t vbytes = (n_rows + 7) / 8;
    DevBuf stats(c, 32);
    for (uint32_t a = 0; a < n_cols; ++a) {
        const hb_column& in = cols[a];
        Column& col = rel->cols[a];
        col.type = in.type;
        if (in.type == HB_COL_STRING) {
            if (!in.offsets) fail(HB_ERR_INVALID_ARG, "string column " + std::to_string(a) + " has no offsets");
            uint64_t total;
            if (on_device) {
                total = read1(c, in.offsets + n_rows);
            } else {
                if (in.offsets[0] != 0) fail(HB_ERR_INVALID_ARG, "string offsets must start at 0");
                for (uint32_t r = 0; r < n_rows; ++r)
                    if (in.offsets[r + 1] < in.offsets[r])
                        fail(HB_ERR_INVALID_ARG, "string offsets of column " + std::to_string(a) + " decrease");
                total = in.offsets[n_rows];
            }
            if (total > 0 && !in.bytes) fail(HB_ERR_INVALID_ARG, "string column " + std::to_string(a) + " has no bytes");
            col.off.alloc(c, sizeof(uint64_t) * ((size_t)n_rows + 1));
            HB_HIP(hipMemcpyAsync(col.off.get(), in.offsets, sizeof(uint64_t) * ((size_t)n_rows + 1), kind, c->stream));
            col.bytes.alloc(c, total + 16);
            if (total) HB_HIP(hipMemcpyAsync(col.bytes.get(), in.bytes, total, kind, c->stream));
            zero(c, stats.get(), 32);
            uint32_t* d_max = stats.as<uint32_t>();
            unsigned long long* d_total = (unsigned long long*)(stats.as<uint8_t>() + 8);
            uint32_t* d_bad = (uint32_t*)(stats.as<uint8_t>() + 16);
            HB_HIP(launch_string_stats(col.off.as<uint64_t>(), n_rows, d_max, d_total, d_bad, c->stream));
            uint32_t h[6];
            HB_HIP(hipMemcpyAsync(h, stats.get(), 24, hipMemcpyDeviceToHost, c->stream));
            c->sync();
            if (h[4]) fail(HB_ERR_INVALID_ARG, "string offsets of column " + std::to_string(a) + " are invalid");
            col.max_len = h[0];
            uint64_t tot;
            std::memcpy(&tot, &h[2], 8);
            col.mean_len = (double)tot / (double)n_rows;
        } else if (in.type == HB_COL_CATEGORICAL || in.type == HB_COL_INT64) {
            if (!in.values) fail(HB_ERR_INVALID_ARG, "column " + std::to_string(a) + " has no values");
            col.values.alloc(c, sizeof(int64_t) * n_rows);
            HB_HIP(hipMemcpyAsync(col.values.get(), in.values, sizeof(int64_t) * n_rows, kind, c->stream));
        } else {
            fail(HB_ERR_INVALID_ARG, "column " + std::to_string(a) + " has an unknown type");
        }
        if (in.valid) {
            col.valid.alloc(c, vbytes);
            HB_HIP(hipMemcpyAsync(col.valid.get(), in.valid, vbytes, kind, c->stream));
        }
    }
    rel->h_cols.resize(n_cols);
    for (uint32_t a = 0; a < n_cols; ++a) {
        const Column& col = rel->cols[a];
        ColDev d{};
        d.type = col.type;
        d.max_len = col.max_len;
        d.off = col.off.as<uint64_t>();
        d.bytes = col.bytes.as<uint8_t>();
        d.values = col.values.as<int64_t>();
        d.valid = col.valid.as<uint8_t>();
        rel->h_cols[a] = d;
    }
    rel->d_cols.alloc(c, sizeof(ColDev) * n_cols);
    HB_HIP(hipMemcpyAsync(rel->d_cols.get(), rel->h_cols.data(), sizeof(ColDev) * n_cols, hipMemcpyHostToDevice,
                          c->stream));
    c->sync();
    rel->id = c->next_id++;
    *rel_id = rel->id;
    c->rels[rel->id] = std::move(rel);
}

// ------------------------------------------------------------ gram index

// Bytes of a string column's arena (allocated with 16 bytes of padding).
static double arena_bytes(const Column& col) { return col.bytes.size() >= 16 ? (double)(col.bytes.size() - 16) : 0.0; }

static GramIndex& gram_index(Ctx* c, Relation& rel, uint32_t attr, uint32_t q) {
    auto key = std::make_pair(attr, q);
    auto it = rel.grams.find(key);
    if (it != rel.grams.end()) return it->second;
    if (c->arena) fail(HB_ERR_STATE, "internal: q-gram index built inside an allocation-free call");
    const uint32_t n = rel.n_rows;
    GramIndex g;
    g.attr = attr;
    g.q = q;
    DevBuf slots(c, sizeof(uint64_t) * ((size_t)n + 1));
    g.off.alloc(c, sizeof(uint64_t) * ((size_t)n + 1));
    const ColDev* dcol = rel.d_cols.as<ColDev>() + attr;
    // algorithmic bytes: T string bytes, W <= T windows (codes), n rows
    const double T = arena_bytes(rel.cols[attr]), nr = (double)n + 1.0;
    const double W = std::max(0.0, T - (double)(q - 1) * (double)n);
    c->timed("gram_slots", [&] { return launch_gram_slots(dcol, n, q, slots.as<uint64_t>(), c->stream); }, 16.0 * nr);
    zero(c, slots.as<uint64_t>() + n, sizeof(uint64_t));
    DevBuf tmp(c, sizeof(uint64_t) * scan_tmp_elems((size_t)n + 1));
    c->timed("gram_slots", [&] {
        return launch_exclusive_scan_u64(slots.as<uint64_t>(), g.off.as<uint64_t>(), (size_t)n + 1, tmp.as<uint64_t>(),
                                         c->stream);
    }, 16.0 * nr);
    // no read-back: a row reserves at most one slot per byte, so the
    // column's byte count bounds the codes, and its longest row's window
    // count bounds every row's distinct codes (the LDS sizing needs no more)
    const uint32_t ml = rel.cols[attr].max_len;
    const uint32_t max_windows = ml >= q ? ml - q + 1 : 1;
    g.codes.alloc(c, sizeof(uint32_t) * (rel.cols[attr].bytes.size() + 1));
    g.cnt.alloc(c, sizeof(uint32_t) * n);
    g.flags.alloc(c, n);
    // long rows get a 256-bit signature: with ~100 codes a 64-bit one is
    // mostly ones and the Jaccard filter bound barely prunes
    g.sig_words = max_windows > 64 ? kLongSigWords : 1;
    g.sig.alloc(c, sizeof(uint64_t) * n * g.sig_words);
    c->timed("gram_build", [&] {
        return launch_gram_build(dcol, n, q, g.off.as<uint64_t>(), g.codes.as<uint32_t>(), g.cnt.as<uint32_t>(),
                                 g.flags.as<uint8_t>(), g.sig.as<uint64_t>(), max_windows, c->stream);
    }, 16.0 * nr + T + 4.0 * W + 5.0 * (double)n + 8.0 * g.sig_words * (double)n);
    g.max_cnt = max_windows;
    auto res = rel.grams.emplace(key, std::move(g));
    return res.first->second;
}

// ------------------------------------------------------------ compile

static bool same_pred(const hb_pred& a, const hb_pred& b) {
    if (a.op != b.op || a.attr != b.attr) return false;
    switch (a.op) {
    case HB_ED_LE: return a.k == b.k;
    case HB_JACCARD_GE: return a.q == b.q && a.num == b.num && a.den == b.den;
    case HB_ABSDIFF_LE: return a.d == b.d;
    case HB_EQ_CONST: return a.side == b.side && a.c == b.c;
    case HB_EQ_CROSS: return a.attr_b == b.attr_b;
    case HB_ED_CROSS_LE: return a.attr_b == b.attr_b && a.k == b.k;
    case HB_JACCARD_CROSS_GE:
    case HB_CONTAIN_GE: return a.attr_b == b.attr_b && a.q == b.q && a.num == b.num && a.den == b.den;
    default: return true;
    }
}

static double pred_cost(const Relation& rel, const hb_pred& p) {
    const Column& col = rel.cols[p.attr];
    const double L = col.mean_len;
    switch (p.op) {
    case HB_EQ: return col.type == HB_COL_STRING ? 1.0 + L / 16.0 : 1.0;
    case HB_ABSDIFF_LE: return 1.5;
    case HB_ED_LE: return 4.0 + 17.0 * L * std::max(1.0, std::ceil(L / 64.0));
    case HB_JACCARD_GE: return 4.0 + 6.0 * std::max(1.0, L - (double)p.q + 1.0);
    case HB_EQ_CONST: return 1.0;
    case HB_EQ_CROSS: return 2.0;   // one compare per valuation
    case HB_ED_CROSS_LE: {          // one Myers run per valuation
        const double M = std::max(L, rel.cols[p.attr_b].mean_len);
        return 2.0 * (4.0 + 17.0 * M * std::max(1.0, std::ceil(M / 64.0)));
    }
    case HB_JACCARD_CROSS_GE:
    case HB_CONTAIN_GE: {           // one list merge per valuation
        const double M = std::max(L, rel.cols[p.attr_b].mean_len);
        return 2.0 * (4.0 + 6.0 * std::max(1.0, M - (double)p.q + 1.0));
    }
    }
    return 1.0;
}

static const uint64_t* char_signature(Ctx* c, Relation& rel, uint32_t attr);

// ------------------------------------------------------------ per-pair cost network

static uint32_t align_up(uint32_t v, uint32_t a) { return (v + a - 1) / a * a; }

constexpr uint32_t kMaxPairSamples = 65536;

// The per-pair network's view of the rule set's distinct predicates
// (Section 4.2, "Evaluation cost"): each compares one attribute of both
// tuples; the q-gram indexes are the relation's (built by compile).
static PairParams pair_params(Ctx* c, Relation& rel, const RuleSet& rs, uint32_t samples, uint64_t seed) {
    PairParams P{};
    if (rs.distinct.size() > (size_t)kMaxSpecs) fail(HB_ERR_LIMIT, "more than 64 distinct predicates");
    std::vector<std::pair<uint32_t, uint32_t>> grams;
    uint32_t lds = kPairLdsGrams + 16;
    for (size_t x = 0; x < rs.distinct.size(); ++x) {
        const hb_pred& d = rs.distinct[x];
        PairSpec& sp = P.spec[x];
        sp.attr = d.attr;
        const bool str = rel.cols[d.attr].type == HB_COL_STRING;
        if (d.op == HB_EQ || (d.op == HB_EQ_CROSS && d.attr_b == d.attr)) {
            sp.kind = str ? PK_STRING_EQ : PK_VALUE_EQ;
        } else if (d.op == HB_ABSDIFF_LE) {
            sp.kind = PK_ABSDIFF;
            sp.d = d.d;
        } else if (d.op == HB_ED_LE) {
            sp.kind = PK_EDIT;
            sp.k = (uint32_t)d.k;
        } else if (d.op == HB_JACCARD_GE) {
            sp.kind = PK_JACCARD;
            sp.q = d.q;
            sp.num = d.num;
            sp.den = d.den;
            auto key = std::make_pair(d.attr, d.q);
            auto it = std::find(grams.begin(), grams.end(), key);
            if (it == grams.end()) {
                if (grams.size() == (size_t)kMaxGramRes) fail(HB_ERR_LIMIT, "more than 8 q-gram attributes");
                grams.push_back(key);
                it = grams.end() - 1;
            }
            sp.gram = (uint8_t)(it - grams.begin());
            P.gram[sp.gram] = gram_index(c, rel, d.attr, d.q).dev();
            lds = std::max<uint32_t>(lds, kPairLdsGrams + (uint32_t)align_up(std::max<uint32_t>(
                                                               P.gram[sp.gram].max_cnt, 1) * 4, 16));
        } else {
            fail(HB_ERR_INVALID_ARG, "the per-pair cost network takes predicates that compare one attribute of "
                                     "both tuples (t.A = s.A, t.A ~ s.A) only");
        }
    }
    if (lds > c->lds_limit) fail(HB_ERR_LIMIT, "the per-pair logging pass exceeds the device's LDS");
    P.cols = rel.d_cols.as<ColDev>();
    P.n_spec = (uint32_t)rs.distinct.size();
    P.samples = rel.n_rows >= 2 ? samples : 0;   // one tuple: no pairs
    P.n_rows = rel.n_rows;
    P.seed = seed;
    P.lds_bytes = lds;
    return P;
}

// Estimated costs (Section 4.2, "Estimated cost"): per predicate, the sum
// of the per-pair network's estimates over the sampled pairs of D x D,
// normalised by the largest sum into (0, 1] (each kept at or above 2^-20 of
// it; every cost 1 when all sums are zero or there are no pairs).  One
// synchronisation: compile reads the sums back.
static void pair_net_costs(Ctx* c, Relation& rel, RuleSet& rs) {
    if (!c->pair_model.ready)
        fail(HB_ERR_STATE, "the per-pair cost estimate needs a per-pair model (hb_costmodel_select, then train)");
    PairParams P = pair_params(c, rel, rs, c->cost_samples, c->cost_seed);
    const size_t np = rs.distinct.size();
    const size_t rows = (size_t)P.n_spec * P.samples;
    std::vector<double> sums(np, 0.0);
    if (rows) {
        DevBuf feat(c, sizeof(float) * kFeatures * rows), y(c, sizeof(float) * 2 * rows), dsum(c, sizeof(double) * np);
        P.features = feat.as<float>();
        P.y = y.as<float>();
        P.sums = dsum.as<double>();
        c->timed("pair_cost", [&] { return launch_pair_features(P, c->stream); });
        c->timed("pair_cost", [&] {
            return launch_mlp_forward(c->pair_model.params.as<float>(), P.features, rows, P.y, c->stream);
        });
        c->timed("pair_cost", [&] { return launch_pair_sum(P, c->stream); });
        HB_HIP(hipMemcpyAsync(sums.data(), P.sums, sizeof(double) * np, hipMemcpyDeviceToHost, c->stream));
        c->sync();
    }
    double top = 0.0;
    for (double v : sums) top = std::max(top, v);
    for (size_t p = 0; p < np; ++p) rs.cost[p] = top > 0.0 ? std::max(sums[p], top * 0x1p-20) / top : 1.0;
}

static void pair_log_collect(Ctx* c, uint32_t rel_id, uint32_t rs_id, uint32_t samples, uint64_t seed,
                             float* features, float* labels, uint32_t* pairs, uint64_t cap, uint64_t* n_rows) {
    Relation& rel = get_rel(c, rel_id);
    RuleSet& rs = get_rs(c, rs_id, rel_id);
    if (!n_rows) fail(HB_ERR_INVALID_ARG, "NULL n_rows");
    if (samples == 0 || samples > kMaxPairSamples) fail(HB_ERR_INVALID_ARG, "samples must be in [1, 65536]");
    PairParams P = pair_params(c, rel, rs, samples, seed);
    const size_t rows = (size_t)P.n_spec * P.samples;
    *n_rows = rows;
    if (cap < rows) fail(HB_ERR_CAPACITY, "row capacity " + std::to_string(cap) + " < " + std::to_string(rows));
    if (rows == 0) return;
    DevBuf feat(c, sizeof(float) * kFeatures * rows), sat(c, rows), cyc(c, sizeof(unsigned long long) * rows);
    DevBuf pr(c, sizeof(uint32_t) * 2 * (size_t)P.samples);
    P.features = feat.as<float>();
    P.sat = sat.as<uint8_t>();
    P.cycles = cyc.as<unsigned long long>();
    P.pairs = pr.as<uint32_t>();
    c->timed("log", [&] { return launch_pair_log(P, c->stream); });
    std::vector<uint8_t> hs(rows);
    std::vector<unsigned long long> hc(rows);
    if (features)
        HB_HIP(hipMemcpyAsync(features, P.features, sizeof(float) * kFeatures * rows, hipMemcpyDeviceToHost, c->stream));
    if (pairs)
        HB_HIP(hipMemcpyAsync(pairs, P.pairs, sizeof(uint32_t) * 2 * (size_t)P.samples, hipMemcpyDeviceToHost,
                              c->stream));
    HB_HIP(hipMemcpyAsync(hs.data(), P.sat, rows, hipMemcpyDeviceToHost, c->stream));
    HB_HIP(hipMemcpyAsync(hc.data(), P.cycles, sizeof(unsigned long long) * rows, hipMemcpyDeviceToHost, c->stream));
    c->sync();
    if (labels)
        for (size_t r = 0; r < rows; ++r) {
            labels[2 * r] = (float)hs[r];
            labels[2 * r + 1] = (float)(std::log2(1.0 + (double)hc[r]) / 16.0);
        }
}

static void compile_rules(Ctx* c, uint32_t rel_id, uint32_t n_rules, const hb_rule* rules, uint32_t* ruleset_id) {
    Relation& rel = get_rel(c, rel_id);
    if (!rules || !ruleset_id) fail(HB_ERR_INVALID_ARG, "NULL argument");
    if (n_rules == 0) fail(HB_ERR_INVALID_ARG, "empty rule set");
    if (n_rules > HB_MAX_RULES) fail(HB_ERR_LIMIT, "more than 64 rules");
    auto rs = std::make_unique<RuleSet>();
    rs->rel_id = rel_id;
    for (uint32_t r = 0; r < n_rules; ++r) {
        const hb_rule& rule = rules[r];
        if (rule.n_preds == 0 || !rule.preds) fail(HB_ERR_INVALID_ARG, "rule " + std::to_string(r) + " is empty");
        if (rule.n_preds > HB_MAX_RULE_PREDS) fail(HB_ERR_LIMIT, "rule " + std::to_string(r) + " has more than 10 predicates");
        std::vector<uint32_t> ids;
        int64_t key = -1;
        for (uint32_t x = 0; x < rule.n_preds; ++x) {
            hb_pred p = rule.preds[x];
            const std::string where = "rule " + std::to_string(r) + " predicate " + std::to_string(x);
            if (p.attr >= rel.n_cols) fail(HB_ERR_INVALID_ARG, where + ": attribute out of range");
            const int32_t t = rel.cols[p.attr].type;
            switch (p.op) {
            case HB_EQ:
                if (key < 0 && t != HB_COL_STRING) key = p.attr;
                break;
            case HB_ED_LE:
                if (t != HB_COL_STRING) fail(HB_ERR_TYPE, where + ": edit distance needs a string attribute");
                if (p.k < 0 || p.k > HB_MAX_ED_K) fail(HB_ERR_INVALID_ARG, where + ": k must be in [0, 255]");
                if (rel.cols[p.attr].max_len > HB_MAX_ED_LEN)
                    fail(HB_ERR_LIMIT, where + ": strings longer than 256 bytes");
                break;
            case HB_JACCARD_GE:
                if (t != HB_COL_STRING) fail(HB_ERR_TYPE, where + ": Jaccard needs a string attribute");
                if (p.q < 1 || p.q > HB_MAX_Q) fail(HB_ERR_INVALID_ARG, where + ": q must be in [1, 4]");
                if (p.den == 0 || p.num > p.den) fail(HB_ERR_INVALID_ARG, where + ": need 0 <= num <= den, den > 0");
                {   // lowest terms (equal thresholds dedup; the bounds below use 32-bit products)
                    uint32_t a = p.num, b = p.den;
                    while (b) { const uint32_t t2 = a % b; a = b; b = t2; }
                    if (a > 1) { p.num /= a; p.den /= a; }
                }
                if (p.den > HB_MAX_JACCARD_DEN) fail(HB_ERR_LIMIT, where + ": threshold denominator above 2^18");
                if (rel.cols[p.attr].max_len > HB_MAX_GRAM_LEN)
                    fail(HB_ERR_LIMIT, where + ": strings longer than 4096 bytes");
                break;
            case HB_ABSDIFF_LE:
                if (t != HB_COL_INT64) fail(HB_ERR_TYPE, where + ": |a-b| <= d needs an int64 attribute");
                if (p.d < 0) fail(HB_ERR_INVALID_ARG, where + ": d must be >= 0");
                break;
            case HB_EQ_CONST:
                if (t == HB_COL_STRING) fail(HB_ERR_TYPE, where + ": t.A = c needs a categorical or int64 attribute");
                if (p.side != 0 && p.side != 1) fail(HB_ERR_INVALID_ARG, where + ": side must be 0 (t) or 1 (s)");
                rs->ordered = true;
                break;
            case HB_EQ_CROSS:
                if (p.attr_b >= rel.n_cols) fail(HB_ERR_INVALID_ARG, where + ": attribute B out of range");
                if (t == HB_COL_STRING || rel.cols[p.attr_b].type == HB_COL_STRING)
                    fail(HB_ERR_TYPE, where + ": t.A = s.B needs categorical or int64 attributes");
                if (p.attr_b != p.attr) rs->ordered = true;
                break;
            case HB_ED_CROSS_LE:
                if (p.attr_b >= rel.n_cols) fail(HB_ERR_INVALID_ARG, where + ": attribute B out of range");
                if (t != HB_COL_STRING || rel.cols[p.attr_b].type != HB_COL_STRING)
                    fail(HB_ERR_TYPE, where + ": t.A ~ s.B (edit distance) needs string attributes");
                if (p.k < 0 || p.k > HB_MAX_ED_K) fail(HB_ERR_INVALID_ARG, where + ": k must be in [0, 255]");
                if (rel.cols[p.attr].max_len > HB_MAX_ED_LEN || rel.cols[p.attr_b].max_len > HB_MAX_ED_LEN)
                    fail(HB_ERR_LIMIT, where + ": strings longer than 256 bytes");
                if (p.attr_b == p.attr) p.op = HB_ED_LE;   // the plain edit distance
                else rs->ordered = true;
                break;
            case HB_JACCARD_CROSS_GE:
                if (p.attr_b >= rel.n_cols) fail(HB_ERR_INVALID_ARG, where + ": attribute B out of range");
                if (t != HB_COL_STRING || rel.cols[p.attr_b].type != HB_COL_STRING)
                    fail(HB_ERR_TYPE, where + ": t.A ~ s.B (Jaccard) needs string attributes");
                if (p.q < 1 || p.q > HB_MAX_Q) fail(HB_ERR_INVALID_ARG, where + ": q must be in [1, 4]");
                if (p.den == 0 || p.num > p.den) fail(HB_ERR_INVALID_ARG, where + ": need 0 <= num <= den, den > 0");
                {
                    uint32_t a = p.num, b = p.den;
                    while (b) { const uint32_t t2 = a % b; a = b; b = t2; }
                    if (a > 1) { p.num /= a; p.den /= a; }
                }
                if (p.den > HB_MAX_JACCARD_DEN) fail(HB_ERR_LIMIT, where + ": threshold denominator above 2^18");
                if (rel.cols[p.attr].max_len > HB_MAX_GRAM_LEN || rel.cols[p.attr_b].max_len > HB_MAX_GRAM_LEN)
                    fail(HB_ERR_LIMIT, where + ": strings longer than 4096 bytes");
                if (p.attr_b == p.attr) p.op = HB_JACCARD_GE;   // the plain Jaccard
                else rs->ordered = true;
                break;
            case HB_CONTAIN_GE:
                if (p.attr_b >= rel.n_cols) fail(HB_ERR_INVALID_ARG, where + ": attribute B out of range");
                if (t != HB_COL_STRING || rel.cols[p.attr_b].type != HB_COL_STRING)
                    fail(HB_ERR_TYPE, where + ": q-gram containment needs string attributes");
                if (p.q < 1 || p.q > HB_MAX_Q) fail(HB_ERR_INVALID_ARG, where + ": q must be in [1, 4]");
                if (p.den == 0 || p.num > p.den) fail(HB_ERR_INVALID_ARG, where + ": need 0 <= num <= den, den > 0");
                {
                    uint32_t a = p.num, b = p.den;
                    while (b) { const uint32_t t2 = a % b; a = b; b = t2; }
                    if (a > 1) { p.num /= a; p.den /= a; }
                }
                if (p.den > HB_MAX_JACCARD_DEN) fail(HB_ERR_LIMIT, where + ": threshold denominator above 2^18");
                if (rel.cols[p.attr].max_len > HB_MAX_GRAM_LEN || rel.cols[p.attr_b].max_len > HB_MAX_GRAM_LEN)
                    fail(HB_ERR_LIMIT, where + ": strings longer than 4096 bytes");
                rs->ordered = true;   // asymmetric, also on one attribute
                break;
            default:
                fail(HB_ERR_INVALID_ARG, where + ": unknown operator");
            }
            uint32_t id = (uint32_t)rs->distinct.size();
            for (uint32_t y = 0; y < rs->distinct.size(); ++y)
                if (same_pred(rs->distinct[y], p)) { id = y; break; }
            if (id == rs->distinct.size()) {
                if (rs->distinct.size() >= HB_MAX_DISTINCT_PREDS) fail(HB_ERR_LIMIT, "more than 64 distinct predicates");
                hb_pred np = p;
                const bool jac = np.op == HB_JACCARD_GE || np.op == HB_JACCARD_CROSS_GE || np.op == HB_CONTAIN_GE;
                if (np.op != HB_ED_LE && np.op != HB_ED_CROSS_LE) np.k = 0;
                if (!jac) { np.q = 0; np.num = 0; np.den = 1; }
                if (np.op != HB_ABSDIFF_LE) np.d = 0;
                if (np.op != HB_EQ_CROSS && np.op != HB_ED_CROSS_LE && np.op != HB_JACCARD_CROSS_GE &&
                    np.op != HB_CONTAIN_GE)
                    np.attr_b = 0;
                if (np.op != HB_EQ_CONST) { np.side = 0; np.c = 0; }
                rs->distinct.push_back(np);
            }
            if (std::find(ids.begin(), ids.end(), id) == ids.end()) ids.push_back(id);
        }
        if (key < 0) fail(HB_ERR_UNBLOCKABLE, "rule " + std::to_string(r) + " has no equality on a categorical/int64 attribute");
        if (std::find(rs->keys.begin(), rs->keys.end(), (uint32_t)key) == rs->keys.end()) rs->keys.push_back((uint32_t)key);
        rs->rules.push_back(ids);
    }
    if (rs->keys.size() > HB_MAX_KEYS) fail(HB_ERR_LIMIT, "more than 4 distinct blocking keys");

    // q-gram indexes, selectivity (LSH evenness) and cost estimates
    const size_t np = rs->distinct.size();
    rs->sp.resize(np);
    rs->cost.resize(np);
    rs->buckets.assign(np, std::vector<uint64_t>(kLshK, 0));
    rs->bucket_n.assign(np, 0);
    DevBuf hist(c, sizeof(unsigned long long) * kLshK * np);
    zero(c, hist.get(), hist.size());
    // the LSH hash depends on (attribute, operator, q or d), not on the
    // threshold: predicates that share those share one histogram
    std::vector<size_t> same(np);
    for (size_t p = 0; p < np; ++p) {
        const hb_pred& pr = rs->distinct[p];
        same[p] = p;
        for (size_t y = 0; y < p; ++y) {
            const hb_pred& py = rs->distinct[y];
            const bool qdep = pr.op == HB_JACCARD_GE || pr.op == HB_JACCARD_CROSS_GE || pr.op == HB_CONTAIN_GE;
            if (py.attr == pr.attr && py.op == pr.op && (!qdep || py.q == pr.q) &&
                (pr.op != HB_ABSDIFF_LE || py.d == pr.d)) { same[p] = y; break; }
        }
        const bool grams = pr.op == HB_JACCARD_GE || pr.op == HB_JACCARD_CROSS_GE || pr.op == HB_CONTAIN_GE;
        if (grams) gram_index(c, rel, pr.attr, pr.q);
        if (pr.op == HB_JACCARD_CROSS_GE || pr.op == HB_CONTAIN_GE) gram_index(c, rel, pr.attr_b, pr.q);
        if (same[p] != p) continue;
        // t.A = c and t.A = s.B take the equality hash of A, t.A ~ s.B the
        // edit-distance or q-gram hash of A: their sp is that of the
        // predicate on A alone (it orders predicates only)
        const int op = pr.op == HB_ED_LE || pr.op == HB_ED_CROSS_LE ? 1
                     : grams ? 2 : pr.op == HB_ABSDIFF_LE ? 3 : 0;
        const Column& lc = rel.cols[pr.attr];
        const double lsh_bytes = lc.type == HB_COL_STRING ? 8.0 * ((double)rel.n_rows + 1.0) + arena_bytes(lc)
                                                         : 8.0 * (double)rel.n_rows;
        c->timed("lsh", [&] {
            return launch_lsh_hist(rel.d_cols.as<ColDev>() + pr.attr, rel.n_rows, op, pr.q, pr.d,
                                   hist.as<unsigned long long>() + p * kLshK, c->stream);
        }, lsh_bytes);
    }
    std::vector<uint64_t> h(kLshK * np);
    HB_HIP(hipMemcpyAsync(h.data(), hist.get(), sizeof(uint64_t) * h.size(), hipMemcpyDeviceToHost, c->stream));
    c->sync();
    for (size_t p = 0; p < np; ++p)
        if (same[p] != p) std::copy_n(h.begin() + same[p] * kLshK, kLshK, h.begin() + p * kLshK);
    double cmax = 0.0;
    for (size_t p = 0; p < np; ++p) {
        unsigned __int128 s2 = 0;
        uint64_t n = 0;
        for (int b = 0; b < kLshK; ++b) {
            uint64_t v = h[p * kLshK + b];
            rs->buckets[p][b] = v;
            n += v;
            s2 += (unsigned __int128)v * v;
        }
        rs->bucket_n[p] = n;
        if (n == 0) {
            rs->sp[p] = 0.0;
        } else {
            // sp = sqrt((k * sum b^2 - n^2) / (n^2 (k - 1)))
            unsigned __int128 num = (unsigned __int128)kLshK * s2 - (unsigned __int128)n * n;
            unsigned __int128 den = (unsigned __int128)n * n * (kLshK - 1);
            rs->sp[p] = std::sqrt((double)num / (double)den);
        }
        rs->cost[p] = pred_cost(rel, rs->distinct[p]);
        cmax = std::max(cmax, rs->cost[p]);
    }
    for (size_t p = 0; p < np; ++p) rs->cost[p] /= cmax;
    if (c->cost_source == HB_COST_PAIR_NET) pair_net_costs(c, rel, *rs);
    // the character signatures every string step reads, built here with the
    // q-gram indexes so that matching only reads per-relation indexes
    for (const hb_pred& d : rs->distinct) {
        if ((d.op == HB_EQ && rel.cols[d.attr].type == HB_COL_STRING) || d.op == HB_ED_LE || d.op == HB_ED_CROSS_LE)
            char_signature(c, rel, d.attr);
        if (d.op == HB_ED_CROSS_LE) char_signature(c, rel, d.attr_b);
    }
    rs->id = c->next_id++;
    *ruleset_id = rs->id;
    c->rulesets[rs->id] = std::move(rs);
}

// ------------------------------------------------------------ partition

// Rows valid on every attribute in `attrs`, sorted by those attributes
// (lexicographically, in the given order); returns the row count.
static uint32_t sort_rows_by(Ctx* c, Relation& rel, const std::vector<uint32_t>& attrs, DevBuf& rows_out) {
    const uint32_t n = rel.n_rows;
    DevBuf d_attrs(c, sizeof(uint32_t) * attrs.size());
    HB_HIP(hipMemcpyAsync(d_attrs.get(), attrs.data(), sizeof(uint32_t) * attrs.size(), hipMemcpyHostToDevice, c->stream));
    DevBuf flags(c, sizeof(uint32_t) * n), dest(c, sizeof(uint32_t) * n);
    HB_HIP(launch_multi_valid_flags(rel.d_cols.as<ColDev>(), d_attrs.as<uint32_t>(), (uint32_t)attrs.size(), n,
                                    flags.as<uint32_t>(), c->stream));
    DevBuf stmp(c, sizeof(uint32_t) * scan_tmp_elems(n));
    HB_HIP(launch_exclusive_scan_u32(flags.as<uint32_t>(), dest.as<uint32_t>(), n, stmp.as<uint32_t>(), c->stream));
    // every attribute's min / max (they size the radix passes) is read back
    // with the row count, in one synchronisation
    const size_t na = attrs.size();
    DevBuf mm(c, 32 * na);
    std::vector<unsigned long long> init(4 * na, 0ull);
    for (size_t x = 0; x < na; ++x) init[4 * x] = ~0ull;
    HB_HIP(hipMemcpyAsync(mm.get(), init.data(), 32 * na, hipMemcpyHostToDevice, c->stream));
    for (size_t x = 0; x < na; ++x) {
        uint8_t* e = mm.as<uint8_t>() + 32 * x;
        HB_HIP(launch_minmax_u64(rel.cols[attrs[x]].values.as<int64_t>(), rel.cols[attrs[x]].valid.as<uint8_t>(), n,
                                 (unsigned long long*)e, (unsigned long long*)(e + 8), (unsigned int*)(e + 16),
                                 c->stream));
    }
    std::vector<unsigned long long> mmh(4 * na);
    HB_HIP(hipMemcpyAsync(mmh.data(), mm.get(), 32 * na, hipMemcpyDeviceToHost, c->stream));
    uint32_t last[2];
    HB_HIP(hipMemcpyAsync(&last[0], dest.as<uint32_t>() + n - 1, 4, hipMemcpyDeviceToHost, c->stream));
    HB_HIP(hipMemcpyAsync(&last[1], flags.as<uint32_t>() + n - 1, 4, hipMemcpyDeviceToHost, c->stream));
    c->sync();
    const uint32_t nv = last[0] + last[1];
    rows_out.alloc(c, sizeof(uint32_t) * (nv + 1));
    if (nv == 0) return 0;
    HB_HIP(launch_compact_rows(flags.as<uint32_t>(), dest.as<uint32_t>(), n, rows_out.as<uint32_t>(), c->stream));
    DevBuf keys(c, sizeof(uint64_t) * nv), keys_alt(c, sizeof(uint64_t) * nv), rows_alt(c, sizeof(uint32_t) * nv);
    DevBuf rtmp(c, radix_tmp_bytes(nv));
    // least significant attribute first (LSD over attributes)
    for (size_t x = na; x-- > 0;) {
        const uint32_t a = attrs[x];
        const unsigned long long lo = mmh[4 * x], hi = mmh[4 * x + 1];
        HB_HIP(launch_gather_key(rel.d_cols.as<ColDev>(), a, lo, rows_out.as<uint32_t>(), nv, keys.as<uint64_t>(),
                                 c->stream));
        std::vector<int> sh = shifts_for_bits(bit_width(hi - lo), 0);
        bool in_alt = false;
        // per 8-bit pass: the histogram reads the keys, the scatter reads
        // and writes keys and row ids
        c->timed("partition_sort", [&] {
            return radix_sort_pairs(keys.as<uint64_t>(), rows_out.as<uint32_t>(), keys_alt.as<uint64_t>(),
                                    rows_alt.as<uint32_t>(), nv, sh.data(), (int)sh.size(), rtmp.get(), &in_alt,
                                    c->stream);
        }, 32.0 * (double)nv * (double)sh.size());
        if (in_alt) HB_HIP(hipMemcpyAsync(rows_out.get(), rows_alt.get(), sizeof(uint32_t) * nv,
                                          hipMemcpyDeviceToDevice, c->stream));
    }
    return nv;
}

// Groups of equal values over `attrs` among sorted rows: group starts.
static uint32_t group_rows(Ctx* c, Relation& rel, const std::vector<uint32_t>& attrs, const DevBuf& rows, uint32_t nv,
                           DevBuf& gstart) {
    DevBuf d_attrs(c, sizeof(uint32_t) * attrs.size());
    HB_HIP(hipMemcpyAsync(d_attrs.get(), attrs.data(), sizeof(uint32_t) * attrs.size(), hipMemcpyHostToDevice, c->stream));
    DevBuf head(c, sizeof(uint32_t) * nv), gid(c, sizeof(uint32_t) * nv);
    HB_HIP(launch_group_heads(rel.d_cols.as<ColDev>(), d_attrs.as<uint32_t>(), (uint32_t)attrs.size(),
                              rows.as<uint32_t>(), nv, head.as<uint32_t>(), c->stream));
    DevBuf stmp(c, sizeof(uint32_t) * scan_tmp_elems(nv));
    HB_HIP(launch_exclusive_scan_u32(head.as<uint32_t>(), gid.as<uint32_t>(), nv, stmp.as<uint32_t>(), c->stream));
    uint32_t last[2];
    HB_HIP(hipMemcpyAsync(&last[0], gid.as<uint32_t>() + nv - 1, 4, hipMemcpyDeviceToHost, c->stream));
    HB_HIP(hipMemcpyAsync(&last[1], head.as<uint32_t>() + nv - 1, 4, hipMemcpyDeviceToHost, c->stream));
    c->sync();
    const uint32_t ng = last[0] + last[1];
    gstart.alloc(c, sizeof(uint32_t) * ng);
    HB_HIP(launch_group_sizes(head.as<uint32_t>(), gid.as<uint32_t>(), nv, ng, gstart.as<uint32_t>(), c->stream));
    return ng;
}

// Consecutive blocks of at most kPackRows rows (in position order, lone rows
// between them included) are packed into windows of at most kTile
// positions, one tile each: a wave batch then serves several small blocks,
// each pair masked to its own block, where it served one.  Returns false
// (nothing changed) when no window would hold two blocks; otherwise
// replaces the partition's tile table by one over the units.
static bool pack_small_blocks(Ctx* c, Partition& P) {
    const uint32_t nb = P.n_blocks;
    if (!c->pack_small_blocks || nb < 2) return false;
    // the blocks under a tile wide hold one tile each: packing can pay only
    // when they are a sizeable share of the tiles
    if ((double)(nb - P.n_big) < 0.25 * (double)P.n_tiles) return false;
    std::vector<uint32_t> st(nb), sz(nb);
    HB_HIP(hipMemcpyAsync(st.data(), P.blk_start.get(), sizeof(uint32_t) * nb, hipMemcpyDeviceToHost, c->stream));
    HB_HIP(hipMemcpyAsync(sz.data(), P.blk_size.get(), sizeof(uint32_t) * nb, hipMemcpyDeviceToHost, c->stream));
    c->sync();
    std::vector<uint32_t> us, usz, ub;
    std::vector<uint64_t> ubd;
    uint32_t packed = 0;
    for (uint32_t i = 0; i < nb;) {
        uint32_t j = i + 1;
        if (sz[i] <= kPackRows)
            while (j < nb && sz[j] <= kPackRows && st[j] + sz[j] - st[i] <= (uint32_t)kTile) ++j;
        if (j - i >= 2) {
            const uint32_t span = st[j - 1] + sz[j - 1] - st[i];
            // every position ends its block but a block's rows before its last
            uint64_t bounds = span >= 64 ? ~0ull : (1ull << span) - 1ull;
            for (uint32_t k = i; k < j; ++k) {
                const uint32_t o = st[k] - st[i];
                const uint64_t inner = ((1ull << (sz[k] - 1)) - 1ull) << o;   // sz[k] <= kPackRows < 64
                bounds &= ~inner;
            }
            us.push_back(st[i]);
            usz.push_back(span | kPackedUnit);
            ub.push_back(~0u);
            ubd.push_back(bounds);
            ++packed;
        } else {
            us.push_back(st[i]);
            usz.push_back(sz[i]);
            ub.push_back(i);
            ubd.push_back(0ull);
            j = i + 1;
        }
        i = j;
    }
    if (packed == 0) return false;
    const uint32_t nu = (uint32_t)us.size();
    std::vector<uint64_t> prefix(nu + 1, 0);
    for (uint32_t u = 0; u < nu; ++u) {
        const uint64_t T = (usz[u] & kPackedUnit) ? 1 : ((uint64_t)(usz[u] & ~kPackedUnit) + kTile - 1) / kTile;
        prefix[u + 1] = prefix[u] + ((usz[u] & kPackedUnit) ? 1 : T * (T + 1) / 2);
    }
    P.unit_start.alloc(c, sizeof(uint32_t) * nu);
    P.unit_size.alloc(c, sizeof(uint32_t) * nu);
    P.unit_blk.alloc(c, sizeof(uint32_t) * nu);
    P.unit_bounds.alloc(c, sizeof(uint64_t) * nu);
    P.tile_prefix.alloc(c, sizeof(uint64_t) * (nu + 1));
    HB_HIP(hipMemcpyAsync(P.unit_start.get(), us.data(), sizeof(uint32_t) * nu, hipMemcpyHostToDevice, c->stream));
    HB_HIP(hipMemcpyAsync(P.unit_size.get(), usz.data(), sizeof(uint32_t) * nu, hipMemcpyHostToDevice, c->stream));
    HB_HIP(hipMemcpyAsync(P.unit_blk.get(), ub.data(), sizeof(uint32_t) * nu, hipMemcpyHostToDevice, c->stream));
    HB_HIP(hipMemcpyAsync(P.unit_bounds.get(), ubd.data(), sizeof(uint64_t) * nu, hipMemcpyHostToDevice, c->stream));
    HB_HIP(hipMemcpyAsync(P.tile_prefix.get(), prefix.data(), sizeof(uint64_t) * (nu + 1), hipMemcpyHostToDevice,
                          c->stream));
    P.n_units = nu;
    P.n_packed = packed;
    P.n_tiles = prefix[nu];
    P.tile_blk.alloc(c, sizeof(uint32_t) * P.n_tiles);
    HB_HIP(launch_tile_blocks(P.tile_prefix.as<uint64_t>(), nu, P.n_tiles, P.tile_blk.as<uint32_t>(), c->stream));
    c->sync();   // the host vectors are the copies' sources
    return true;
}

static Partition& key_partition(Ctx* c, Relation& rel, uint32_t attr) {
    auto it = rel.parts.find(attr);
    if (it != rel.parts.end()) return it->second;
    Partition P;
    P.attr = attr;
    std::vector<uint32_t> attrs{attr};
    P.n_valid = sort_rows_by(c, rel, attrs, P.perm);
    P.blk_start.alloc(c, 4);
    P.blk_size.alloc(c, 4);
    P.tile_prefix.alloc(c, 8);
    zero(c, P.tile_prefix.get(), 8);
    if (P.n_valid >= 2) {
        DevBuf gstart;
        const uint32_t ng = group_rows(c, rel, attrs, P.perm, P.n_valid, gstart);
        DevBuf flags(c, sizeof(uint32_t) * ng), dest(c, sizeof(uint32_t) * ng);
        HB_HIP(launch_ge2_flags(gstart.as<uint32_t>(), ng, P.n_valid, flags.as<uint32_t>(), c->stream));
        DevBuf stmp(c, sizeof(uint32_t) * scan_tmp_elems(ng));
        HB_HIP(launch_exclusive_scan_u32(flags.as<uint32_t>(), dest.as<uint32_t>(), ng, stmp.as<uint32_t>(), c->stream));
        uint32_t last[2];
        HB_HIP(hipMemcpyAsync(&last[0], dest.as<uint32_t>() + ng - 1, 4, hipMemcpyDeviceToHost, c->stream));
        HB_HIP(hipMemcpyAsync(&last[1], flags.as<uint32_t>() + ng - 1, 4, hipMemcpyDeviceToHost, c->stream));
        c->sync();
        P.n_blocks = last[0] + last[1];
        P.blk_start.alloc(c, sizeof(uint32_t) * (P.n_blocks + 1));
        P.blk_size.alloc(c, sizeof(uint32_t) * (P.n_blocks + 1));
        DevBuf tiles(c, sizeof(uint64_t) * (P.n_blocks + 1));
        zero(c, tiles.get(), tiles.size());
        DevBuf pairs(c, sizeof(unsigned long long));
        zero(c, pairs.get(), 8);
        HB_HIP(launch_block_table(gstart.as<uint32_t>(), ng, P.n_valid, dest.as<uint32_t>(), P.blk_start.as<uint32_t>(),
                                  P.blk_size.as<uint32_t>(), tiles.as<uint64_t>(), pairs.as<unsigned long long>(),
                                  c->stream));
        P.tile_prefix.alloc(c, sizeof(uint64_t) * (P.n_blocks + 1));
        DevBuf ttmp(c, sizeof(uint64_t) * scan_tmp_elems((size_t)P.n_blocks + 1));
        HB_HIP(launch_exclusive_scan_u64(tiles.as<uint64_t>(), P.tile_prefix.as<uint64_t>(), (size_t)P.n_blocks + 1,
                                         ttmp.as<uint64_t>(), c->stream));
        // blocks holding at least one full row batch
        const uint32_t nb = std::max<uint32_t>(P.n_blocks, 1);
        DevBuf bflags(c, sizeof(uint32_t) * nb), bdest(c, sizeof(uint32_t) * nb);
        DevBuf btmp(c, sizeof(uint32_t) * scan_tmp_elems(nb));
        P.big.alloc(c, sizeof(uint32_t) * nb);
        uint64_t h[2];
        uint32_t hb2[2] = {0, 0};
        if (P.n_blocks) {
            HB_HIP(launch_size_flags(P.blk_size.as<uint32_t>(), P.n_blocks, kTile, bflags.as<uint32_t>(), c->stream));
            HB_HIP(launch_exclusive_scan_u32(bflags.as<uint32_t>(), bdest.as<uint32_t>(), P.n_blocks,
                                             btmp.as<uint32_t>(), c->stream));
            HB_HIP(launch_compact_rows(bflags.as<uint32_t>(), bdest.as<uint32_t>(), P.n_blocks, P.big.as<uint32_t>(),
                                       c->stream));
            HB_HIP(hipMemcpyAsync(&hb2[0], bdest.as<uint32_t>() + P.n_blocks - 1, 4, hipMemcpyDeviceToHost, c->stream));
            HB_HIP(hipMemcpyAsync(&hb2[1], bflags.as<uint32_t>() + P.n_blocks - 1, 4, hipMemcpyDeviceToHost, c->stream));
        }
        HB_HIP(hipMemcpyAsync(&h[0], P.tile_prefix.as<uint64_t>() + P.n_blocks, 8, hipMemcpyDeviceToHost, c->stream));
        HB_HIP(hipMemcpyAsync(&h[1], pairs.get(), 8, hipMemcpyDeviceToHost, c->stream));
        c->sync();
        P.n_tiles = h[0];
        P.pairs = h[1];
        P.n_big = hb2[0] + hb2[1];
        if (P.n_tiles && P.n_tiles <= kMaxTiles) {   // more tiles cannot be matched in one launch
            if (!pack_small_blocks(c, P)) {
                P.tile_blk.alloc(c, sizeof(uint32_t) * P.n_tiles);
                HB_HIP(launch_tile_blocks(P.tile_prefix.as<uint64_t>(), P.n_blocks, P.n_tiles,
                                          P.tile_blk.as<uint32_t>(), c->stream));
            }
        }
    }
    auto res = rel.parts.emplace(attr, std::move(P));
    return res.first->second;
}

static uint64_t composite_pairs(Ctx* c, Relation& rel, const std::vector<uint32_t>& attrs) {
    auto it = rel.composite.find(attrs);
    if (it != rel.composite.end()) return it->second;
    DevBuf rows;
    const uint32_t nv = sort_rows_by(c, rel, attrs, rows);
    uint64_t total = 0;
    if (nv >= 2) {
        DevBuf gstart;
        const uint32_t ng = group_rows(c, rel, attrs, rows, nv, gstart);
        DevBuf pairs(c, 8);
        zero(c, pairs.get(), 8);
        HB_HIP(launch_group_pairs(gstart.as<uint32_t>(), ng, nv, pairs.as<unsigned long long>(), c->stream));
        total = read1(c, pairs.as<unsigned long long>());
    }
    rel.composite[attrs] = total;
    return total;
}

static void partition(Ctx* c, uint32_t rel_id, uint32_t rs_id, uint64_t* n_cand) {
    Relation& rel = get_rel(c, rel_id);
    RuleSet& rs = get_rs(c, rs_id, rel_id);
    for (uint32_t k : rs.keys) key_partition(c, rel, k);
    // distinct pairs sharing at least one key, by inclusion-exclusion
    const size_t K = rs.keys.size();
    __int128 total = 0;
    for (uint32_t mask = 1; mask < (1u << K); ++mask) {
        std::vector<uint32_t> S;
        for (size_t x = 0; x < K; ++x)
            if (mask & (1u << x)) S.push_back(rs.keys[x]);
        uint64_t p = S.size() == 1 ? rel.parts.at(S[0]).pairs : composite_pairs(c, rel, S);
        if (S.size() % 2 == 1) total += p; else total -= p;
    }
    rs.candidates = (uint64_t)total;
    rs.partitioned = true;
    if (n_cand) *n_cand = rs.candidates;
}

// ------------------------------------------------------------ match



static const uint64_t* char_signature(Ctx* c, Relation& rel, uint32_t attr) {
    auto it = rel.char_sig.find(attr);
    if (it != rel.char_sig.end()) return it->second.as<uint64_t>();
    if (c->arena) fail(HB_ERR_STATE, "internal: character signature built inside an allocation-free call");
    DevBuf sig(c, sizeof(uint64_t) * rel.n_rows);
    c->timed("char_sig", [&] { return launch_char_sig(rel.d_cols.as<ColDev>() + attr, rel.n_rows, sig.as<uint64_t>(), c->stream); },
             16.0 * (double)rel.n_rows + arena_bytes(rel.cols[attr]));
    const uint64_t* p = sig.as<uint64_t>();
    rel.char_sig.emplace(attr, std::move(sig));
    return p;
}


// A rule can hold in key `ka`'s blocks unless it needs an earlier key to
// agree (the owner check rules those pairs out).
static bool rule_possible(const Relation& rel, const RuleSet& rs, const std::vector<uint32_t>& preds, size_t ka) {
    for (uint32_t p : preds) {
        const hb_pred& d = rs.distinct[p];
        if (d.op == HB_EQ && rel.cols[d.attr].type != HB_COL_STRING)
            for (size_t x = 0; x < ka; ++x)
                if (rs.keys[x] == d.attr) return false;
    }
    return true;
}

static KeyRes key_resources(const Relation& rel, const RuleSet& rs, size_t ka) {
    KeyRes R;
    const uint32_t key = rs.keys[ka];
    auto res_of = [](std::vector<uint32_t>& v, uint32_t a) {
        auto it = std::find(v.begin(), v.end(), a);
        if (it != v.end()) return (uint32_t)(it - v.begin());
        v.push_back(a);
        return (uint32_t)(v.size() - 1);
    };
    for (size_t x = 0; x < ka; ++x) R.prev.push_back(res_of(R.int_attr, rs.keys[x]));
    std::vector<bool> used(rs.distinct.size(), false);
    for (const auto& rule : rs.rules) {
        if (!rule_possible(rel, rs, rule, ka)) continue;
        R.any_rule = true;
        for (uint32_t p : rule) used[p] = true;
    }
    for (uint32_t p = 0; p < rs.distinct.size(); ++p) {
        if (!used[p]) continue;
        const hb_pred& d = rs.distinct[p];
        const int32_t t = rel.cols[d.attr].type;
        if (d.op == HB_EQ && t != HB_COL_STRING && d.attr == key) continue;
        PredSpec sp{};
        sp.pred = (uint16_t)p;
        switch (d.op) {
        case HB_EQ:
            if (t == HB_COL_STRING) { sp.op = OP_EQ_STR; sp.res = (uint8_t)res_of(R.str_attr, d.attr); }
            else { sp.op = OP_EQ_INT; sp.res = (uint8_t)res_of(R.int_attr, d.attr); }
            break;
        case HB_ABSDIFF_LE:
            sp.op = OP_ABSDIFF;
            sp.res = (uint8_t)res_of(R.int_attr, d.attr);
            sp.param = (uint64_t)d.d;
            break;
        case HB_ED_LE:
            sp.op = OP_ED;
            sp.res = (uint8_t)res_of(R.str_attr, d.attr);
            sp.param = (uint64_t)d.k;
            R.any_ed = true;
            break;
        case HB_EQ_CONST:
            sp.op = OP_CONST;
            sp.res = (uint8_t)res_of(R.int_attr, d.attr);
            sp.aux = (uint8_t)d.side;
            sp.param = (uint64_t)d.c;
            break;
        case HB_EQ_CROSS:
            sp.res = (uint8_t)res_of(R.int_attr, d.attr);
            if (d.attr_b == d.attr) {
                sp.op = OP_EQ_INT;
            } else {
                sp.op = OP_XEQ;
                sp.aux = (uint8_t)res_of(R.int_attr, d.attr_b);
            }
            break;
        case HB_ED_CROSS_LE:   // attr_b != attr (compile turns A = B into HB_ED_LE)
            sp.op = OP_XED;
            sp.res = (uint8_t)res_of(R.str_attr, d.attr);
            sp.aux = (uint8_t)res_of(R.str_attr, d.attr_b);
            sp.param = (uint64_t)d.k;
            R.any_ed = true;
            break;
        case HB_JACCARD_GE: {
            auto gk = std::make_pair(d.attr, d.q);
            auto it = std::find(R.gram_key.begin(), R.gram_key.end(), gk);
            if (it == R.gram_key.end()) { R.gram_key.push_back(gk); sp.res = (uint8_t)(R.gram_key.size() - 1); }
            else sp.res = (uint8_t)(it - R.gram_key.begin());
            sp.op = OP_JAC;
            sp.param = ((uint64_t)d.num << 32) | d.den;
            break;
        }
        case HB_JACCARD_CROSS_GE:     // attr_b != attr (compile turns A = B into HB_JACCARD_GE)
        case HB_CONTAIN_GE: {         // attr_b may equal attr (one gram resource then)
            auto gres = [&](uint32_t attr) -> uint8_t {
                auto gk = std::make_pair(attr, d.q);
                auto it = std::find(R.gram_key.begin(), R.gram_key.end(), gk);
                if (it != R.gram_key.end()) return (uint8_t)(it - R.gram_key.begin());
                R.gram_key.push_back(gk);
                return (uint8_t)(R.gram_key.size() - 1);
            };
            sp.op = d.op == HB_CONTAIN_GE ? OP_XCONT : OP_XJAC;
            sp.res = gres(d.attr);
            sp.aux = gres(d.attr_b);
            sp.param = ((uint64_t)d.num << 32) | d.den;
            break;
        }
        }
        R.specs.push_back(sp);
    }
    if (R.int_attr.size() > (size_t)kMaxIntRes || R.str_attr.size() > (size_t)kMaxStrRes ||
        R.gram_key.size() > (size_t)kMaxGramRes)
        fail(HB_ERR_LIMIT, "rule set reads more than 16 int, 8 string or 8 q-gram attributes");
    return R;
}

// Bytecode of a sequential path for key `ka`: each possible rule becomes its
// cheap steps and filters in path order, then its exact similarity
// predicates in path order, then a checkpoint.  The equality on this key is
// dropped (it holds inside a block).  Consecutive rules whose first step is
// the same cheap step share it, as rules sharing a prefix share the
// execution tree's edge (Section 4.2): the step runs once as a guard, the
// rules run their remaining steps on the pairs that passed it, and a
// group end returns to every pair (not for rule sets that tell t from s).
// `segs` (optional) receives each rule's segment: its first instruction,
// its first-stage steps (in path order) and its guard step.
static std::vector<Instr> emit_code(const Relation& rel, const RuleSet& rs, const std::vector<PathRule>& path,
                                    size_t ka, const KeyRes& R, bool regroup, std::vector<RuleSeg>* segs = nullptr) {
    auto spec_of = [&](uint32_t p) -> const PredSpec* {
        for (const PredSpec& sp : R.specs)
            if (sp.pred == p) return &sp;
        return nullptr;
    };
    struct RuleCode {
        std::vector<Instr> first, verify;
        std::vector<uint32_t> first_preds;
    };
    std::vector<RuleCode> rc;
    for (const PathRule& pr : path) {
        if (!rule_possible(rel, rs, pr.preds, ka)) continue;
        RuleCode r;
        for (uint32_t p : pr.preds) {
            const PredSpec* sp = spec_of(p);
            if (!sp) continue;   // the key's own equality
            Instr in{};
            in.slot = (uint8_t)p;
            in.res = sp->res;
            in.aux = sp->aux;
            in.param = sp->param;
            Instr f = in;
            f.slot = (uint8_t)(64 + p);
            switch (sp->op) {
            case OP_EQ_INT:
            case OP_ABSDIFF:
            case OP_CONST:
            case OP_XEQ:
            case OP_XED:
            case OP_XJAC:
            case OP_XCONT:
                in.op = sp->op;
                r.first.push_back(in);
                break;
            case OP_EQ_STR:
                f.op = OP_EQF;
                in.op = OP_EQ_STR;
                r.first.push_back(f);
                r.verify.push_back(in);
                break;
            case OP_ED:
                f.op = OP_EDF;
                in.op = OP_ED;
                r.first.push_back(f);
                r.verify.push_back(in);
                break;
            default:
                f.op = OP_JACF;
                in.op = OP_JAC;
                r.first.push_back(f);
                r.verify.push_back(in);
                break;
            }
            r.first_preds.push_back(p);
        }
        if (!pr.verify.empty()) {
            // the exact checks in the given order
            std::vector<Instr> ordered;
            for (uint32_t p : pr.verify)
                for (const Instr& in : r.verify)
                    if (in.slot == (uint8_t)p) ordered.push_back(in);
            if (ordered.size() != r.verify.size()) fail(HB_ERR_STATE, "internal: verification order mismatch");
            r.verify.swap(ordered);
        }
        rc.push_back(std::move(r));
    }
    auto same_step = [](const Instr& a, const Instr& b) {
        return a.op == b.op && a.op <= OP_JACF && a.res == b.res && a.aux == b.aux && a.param == b.param;
    };
    // the same cheap step on the same attribute, at any threshold
    auto same_kind = [](const Instr& a, const Instr& b) {
        return a.op == b.op && a.op <= OP_JACF && a.res == b.res && a.aux == b.aux;
    };
    // a passes every pair b passes (a and b of one kind): the larger
    // distance bound, the lower Jaccard threshold num / den
    auto looser = [](const Instr& a, const Instr& b) {
        switch (a.op) {
        case OP_ABSDIFF: return (int64_t)a.param >= (int64_t)b.param;
        case OP_EDF: return (uint32_t)a.param >= (uint32_t)b.param;
        case OP_JACF: {
            const uint64_t na = a.param >> 32, da = a.param & 0xFFFFFFFFu;
            const uint64_t nb = b.param >> 32, db = b.param & 0xFFFFFFFFu;
            return na * db <= nb * da;
        }
        default: return a.param == b.param;
        }
    };
    const bool share = !rs.ordered;
    if (share && regroup) {
        // rules whose first steps are of one kind are placed together, at
        // the first one's place, so that one guard serves them all (the
        // listing is a union over rules, so their order is free)
        std::vector<RuleCode> placed;
        std::vector<bool> used(rc.size(), false);
        for (size_t x = 0; x < rc.size(); ++x) {
            if (used[x]) continue;
            used[x] = true;
            if (rc[x].first.empty() || rc[x].first[0].op > OP_JACF) {
                placed.push_back(std::move(rc[x]));
                continue;
            }
            const Instr head = rc[x].first[0];   // a copy: `placed` grows below
            placed.push_back(std::move(rc[x]));
            for (size_t y = x + 1; y < rc.size(); ++y)
                if (!used[y] && !rc[y].first.empty() && same_kind(rc[y].first[0], head)) {
                    used[y] = true;
                    placed.push_back(std::move(rc[y]));
                }
        }
        rc.swap(placed);
    }
    std::vector<Instr> code;
    if (segs) segs->clear();
    for (size_t x = 0; x < rc.size();) {
        // [x, y): rules sharing their first step; with regrouping, rules
        // whose first steps are of one kind, under a guard at the loosest
        // threshold among them (a pair failing it fails each rule's own)
        size_t y = x + 1;
        size_t owner = x;   // the rule whose first step the guard is
        if (share && !rc[x].first.empty())
            while (y < rc.size() && !rc[y].first.empty() &&
                   (regroup ? same_kind(rc[y].first[0], rc[x].first[0]) : same_step(rc[y].first[0], rc[x].first[0]))) {
                if (looser(rc[y].first[0], rc[owner].first[0]) && !looser(rc[owner].first[0], rc[y].first[0]))
                    owner = y;
                ++y;
            }
        const bool group = y - x >= 2;
        size_t guard_at = 0;
        if (group) {
            Instr g = rc[owner].first[0];
            g.aux = g.op;
            g.op = OP_GUARD;
            guard_at = code.size();
            code.push_back(g);
        }
        for (size_t k = x; k < y; ++k) {
            RuleCode& r = rc[k];
            // a rule whose first step is the guard's does not repeat it
            const size_t skip = group && same_step(r.first[0], rc[owner].first[0]) ? 1 : 0;
            const size_t first = code.size();
            code.insert(code.end(), r.first.begin() + skip, r.first.end());
            code.insert(code.end(), r.verify.begin(), r.verify.end());
            Instr cp{};
            cp.op = OP_CP;
            code.push_back(cp);
            const uint16_t cpi = (uint16_t)(code.size() - 1);
            for (size_t i = first; i < code.size(); ++i) code[i].cp = cpi;
            if (segs) {
                RuleSeg sg;
                sg.start = (uint32_t)first;
                sg.first_preds.assign(r.first_preds.begin() + skip, r.first_preds.end());
                sg.guard_pred = group ? (int)rc[owner].first_preds[0] : -1;
                segs->push_back(std::move(sg));
            }
        }
        if (group) {
            Instr e{};
            e.op = OP_ENDGUARD;
            code.push_back(e);
            code[guard_at].cp = (uint16_t)(code.size() - 1);
        }
        x = y;
    }
    if (code.size() > (size_t)kMaxPlan) fail(HB_ERR_LIMIT, "plan too long");
    return code;
}

// Resources, block-major feature columns and LDS layout of key `ka`'s
// partition (everything but the plan itself).
static bool prepare_key(Ctx* c, Relation& rel, RuleSet& rs, size_t ka, KeyPlan& kp, KeyRes& R, bool count) {
    const uint32_t key = rs.keys[ka];
    R = key_resources(rel, rs, ka);
    if (!R.any_rule) return false;
    const Partition& P = rel.parts.at(key);
    MatchParams& m = kp.mp;
    m.n_int = (uint32_t)R.int_attr.size();
    m.n_str = (uint32_t)R.str_attr.size();
    m.n_gram = (uint32_t)R.gram_key.size();
    m.n_prev = (uint32_t)R.prev.size();
    m.ordered = rs.ordered ? 1u : 0u;
    for (size_t x = 0; x < R.int_attr.size(); ++x) m.int_attr[x] = R.int_attr[x];
    for (size_t x = 0; x < R.prev.size(); ++x) m.prev_res[x] = R.prev[x];
    GatherParams gp{};
    gp.perm = P.perm.as<uint32_t>();
    gp.n = P.n_valid;
    gp.n_int = m.n_int;
    gp.n_str = m.n_str;
    gp.n_gram = m.n_gram;
    for (size_t x = 0; x < R.int_attr.size(); ++x) {
        const Column& col = rel.cols[R.int_attr[x]];
        gp.int_valid[x] = col.valid.size() ? col.valid.as<uint8_t>() : nullptr;
        gp.int_vals[x] = col.values.as<int64_t>();
    }
    for (size_t x = 0; x < R.str_attr.size(); ++x) {
        m.str_attr[x] = R.str_attr[x];
        const Column& col = rel.cols[R.str_attr[x]];
        gp.str_valid[x] = col.valid.size() ? col.valid.as<uint8_t>() : nullptr;
        gp.str_off[x] = col.off.as<uint64_t>();
        gp.csig[x] = char_signature(c, rel, R.str_attr[x]);
    }
    // the pattern-match table covers the longest value an edit distance
    // takes as its pattern (string equality compares bytes, so a long
    // compared-only attribute does not widen it)
    uint32_t ed_words = 1;
    for (const PredSpec& sp : R.specs) {
        if (sp.op != OP_ED && sp.op != OP_XED) continue;
        ed_words = std::max<uint32_t>(ed_words, (rel.cols[R.str_attr[sp.res]].max_len + 63) / 64);
        if (sp.op == OP_XED) ed_words = std::max<uint32_t>(ed_words, (rel.cols[R.str_attr[sp.aux]].max_len + 63) / 64);
    }
    uint32_t gram_cols = 0;   // f64 columns of the q-gram signatures
    for (size_t x = 0; x < R.gram_key.size(); ++x) {
        GramIndex& g = gram_index(c, rel, R.gram_key[x].first, R.gram_key[x].second);
        m.gram[x] = g.dev();
        m.gram[x].sig_col = gram_cols;
        gp.gram_words[x] = g.sig_words;
        gp.gram_col[x] = gram_cols;
        gram_cols += g.sig_words;
        const Column& col = rel.cols[g.attr];
        gp.gram_valid[x] = col.valid.size() ? col.valid.as<uint8_t>() : nullptr;
        gp.gram_cnt[x] = g.cnt.as<uint32_t>();
        gp.gram_flags[x] = g.flags.as<uint8_t>();
        gp.gsig[x] = g.sig.as<uint64_t>();
    }
    m.ed_words = R.any_ed ? ed_words : 0;   // 0: no edit-distance predicate
    const uint32_t n64 = m.n_int + m.n_str + gram_cols, n32 = 2 + m.n_str + 2 * m.n_gram;
    const uint64_t stride = (uint64_t)P.n_valid + kTile;
    gp.stride = stride;
    kp.f64.alloc(c, sizeof(uint64_t) * stride * std::max<uint32_t>(n64, 1));
    kp.f32.alloc(c, sizeof(uint32_t) * stride * n32);
    gp.f64 = kp.f64.as<uint64_t>();
    gp.f32 = kp.f32.as<uint32_t>();
    // reads: the permutation, per int column its value, per string column
    // two offsets and the character signature, per q-gram column count,
    // flag and signature words; writes: every feature column
    const double nvp = (double)P.n_valid;
    const double per_row_in = 8.0 * m.n_int + 24.0 * m.n_str + 5.0 * m.n_gram + 8.0 * gram_cols;
    const double feat_bytes = (double)stride * (8.0 * n64 + 4.0 * n32);
    gp.n64 = n64;
    gp.n32 = n32;
    if (c->arena) {
        // allocation-free: one pass, each column read at the permuted rows
        c->timed("gather", [&] { return launch_gather_features(gp, c->stream); },
                 nvp * (4.0 + per_row_in) + feat_bytes);
    } else {
        // two passes: a read of one feature at a random row moves a whole
        // cache line for 4-8 useful bytes; packed into row records first
        // (sequential reads), the permuted reads move whole records
        gp.n_rows = rel.n_rows;
        gp.rec_words = (uint32_t)align_up(2 * n64 + n32 - 1, 4);
        DevBuf rec(c, sizeof(uint32_t) * (size_t)gp.rec_words * std::max<uint32_t>(rel.n_rows, 1));
        gp.rec = rec.as<uint32_t>();
        const double rec_bytes = 4.0 * gp.rec_words;
        c->timed("gather", [&] { return launch_pack_records(gp, c->stream); },
                 (double)rel.n_rows * (per_row_in + rec_bytes));
        c->timed("gather", [&] { return launch_gather_records(gp, c->stream); },
                 nvp * (4.0 + rec_bytes) + feat_bytes);
    }
    kp.feat_bytes = feat_bytes;

    // LDS of the one-wave workgroup: the pattern-match table, the
    // long-pattern Myers state and the current row's q-gram lists, then the
    // instrumented pass's counters
    uint32_t w = 0;
    m.lds_wave_peq = w;
    if (R.any_ed) w += 256 * ed_words * 8;
    for (uint32_t x = 0; x < m.n_gram; ++x) {
        m.lds_wave_igram[x] = w;
        w += align_up(std::max<uint32_t>(m.gram[x].max_cnt, 1) * 4, 16);
    }
    // last, so that kernels holding the long-pattern state in registers
    // can leave it out
    m.lds_wave_myers = w;
    if (R.any_ed && ed_words >= 2) w += 2 * kMaxEdWords * 64 * 8;
    w = align_up(std::max<uint32_t>(w, 16), 16);
    m.lds_wave_stride = w;
    m.lds_counts = w;
    m.lds_bytes = align_up(w + (count ? kCountSlots * 8 : 0), 16);
    if (m.lds_bytes > c->lds_limit)
        fail(HB_ERR_LIMIT, "the rule set's per-wave working set (" + std::to_string(m.lds_bytes) +
                               " bytes of LDS) exceeds the device limit");

    m.rows = c->rows_per_wave;
    m.sparse_rows = c->sparse_rows;
    {   // no validity bitmap on any attribute a step reads (keys included)
        bool all = true;
        for (uint32_t a : R.int_attr) all = all && rel.cols[a].valid.size() == 0;
        for (uint32_t a : R.str_attr) all = all && rel.cols[a].valid.size() == 0;
        for (const auto& gk : R.gram_key) all = all && rel.cols[gk.first].valid.size() == 0;
        m.all_valid = all ? 1u : 0u;
    }
    m.cols = rel.d_cols.as<ColDev>();
    m.feat.f64 = kp.f64.as<uint64_t>();
    m.feat.f32 = kp.f32.as<uint32_t>();
    m.feat.n = stride;
    m.blk_start = P.blk_start.as<uint32_t>();
    m.blk_size = P.blk_size.as<uint32_t>();
    m.tile_prefix = P.tile_prefix.as<uint64_t>();
    m.tile_blk = P.tile_blk.as<uint32_t>();
    m.unit_start = P.n_units ? P.unit_start.as<uint32_t>() : nullptr;
    m.unit_size = P.n_units ? P.unit_size.as<uint32_t>() : nullptr;
    m.unit_blk = P.n_units ? P.unit_blk.as<uint32_t>() : nullptr;
    m.unit_bounds = P.n_units ? P.unit_bounds.as<uint64_t>() : nullptr;
    m.n_blocks = P.n_blocks;
    m.n_tiles = P.n_tiles;
    if (m.n_tiles > kMaxTiles) fail(HB_ERR_LIMIT, "more than 2^30 - 8 tiles in one key partition");
    return true;
}

// Guards across thresholds (rules regrouped) for the heuristic and learned
// plans; the comparison orders keep their rule order.
static bool regroups(int plan) { return plan == HB_PLAN_HEURISTIC || plan == HB_PLAN_LEARNED; }

static bool build_key_plan(Ctx* c, Relation& rel, RuleSet& rs, int plan, const std::vector<PathRule>& path, size_t ka,
                           KeyPlan& kp, bool count) {
    KeyRes R;
    if (!prepare_key(c, rel, rs, ka, kp, R, count)) return false;
    kp.code = emit_code(rel, rs, path, ka, R, regroups(plan));
    kp.mp.plan_len = (uint32_t)kp.code.size();
    return true;
}

// ------------------------------------------------------------ learned plan

// Features of every (block, predicate) of key `ka` into `feat` (device).
// Features of the listed blocks (all blocks when `blocks` is null).
static void block_features(Ctx* c, const KeyPlan& kp, const KeyRes& R, DevBuf& feat, LearnParams& L,
                           const uint32_t* blocks, uint32_t n_list) {
    if (R.specs.size() > (size_t)kMaxSpecs) fail(HB_ERR_LIMIT, "more than 64 predicates in one partition");
    L = LearnParams{};
    L.mp = kp.mp;
    L.blocks = blocks;
    L.n_list = blocks ? n_list : kp.mp.n_blocks;
    for (size_t x = 0; x < R.specs.size(); ++x) L.spec[x] = R.specs[x];
    L.n_spec = (uint32_t)R.specs.size();
    feat.alloc(c, sizeof(float) * kFeatures * std::max<size_t>((size_t)L.n_list * L.n_spec, 1));
    L.features = feat.as<float>();
    c->timed("block_features", [&] { return launch_block_features(L, c->stream); });
}

static uint32_t next_pow2(uint32_t v) {
    uint32_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

// Learned per-block plans for key `ka`, built on the device without a host
// round trip: block features, cost-model inference (per block and
// predicate: the first plan step's pass rate and the exact check's cycles)
// and the plan-choice kernel, which writes each distinct choice's plan.
// Blocks smaller than one 64 x 64 tile keep the heuristic plan (their
// pairs are few; features and choices would cost more than they save).
static void learned_key_plan(Ctx* c, Relation& rel, RuleSet& rs, size_t ka, KeyPlan& kp, const KeyRes& R,
                             const std::vector<PathRule>& heuristic, uint64_t* n_fallback) {
    if (!c->model.ready) fail(HB_ERR_STATE, "the learned plan needs a cost model (hb_costmodel_train or _set_params)");
    const uint32_t nb = kp.mp.n_blocks;
    const uint32_t ns = (uint32_t)R.specs.size();
    std::vector<RuleSeg> segs;
    kp.code = emit_code(rel, rs, heuristic, ka, R, true, &segs);
    kp.mp.plan_len = (uint32_t)kp.code.size();
    // the partition's rules in heuristic order: where each rule's segment
    // starts, its first-stage steps and the guard step it sits under
    std::vector<int> spec_of(rs.distinct.size(), -1);
    for (uint32_t x = 0; x < ns; ++x) spec_of[R.specs[x].pred] = (int)x;
    PlanChoiceParams C{};
    const uint32_t n_rules = (uint32_t)segs.size();
    const bool ok = nb > 0 && ns > 0 && n_rules > 0 && n_rules <= (uint32_t)kMaxPlanRules;
    if (!ok) {
        *n_fallback += nb;
        return;
    }
    for (uint32_t r = 0; r < n_rules; ++r) {
        const RuleSeg& sg = segs[r];
        if (sg.first_preds.size() > (size_t)kMaxRuleSteps) fail(HB_ERR_LIMIT, "rule with more than 10 steps");
        C.rule_len[r] = (uint8_t)sg.first_preds.size();
        C.rule_seg[r] = (uint16_t)sg.start;
        C.rule_guard[r] = sg.guard_pred < 0 ? (uint8_t)0xFF : (uint8_t)spec_of[sg.guard_pred];
        for (size_t k = 0; k < sg.first_preds.size(); ++k) C.rule_spec[r][k] = (uint8_t)spec_of[sg.first_preds[k]];
    }
    const Partition& part = rel.parts.at(rs.keys[ka]);
    const uint32_t nl = part.n_big;   // blocks with per-block plans; the rest keep slot 0
    kp.blk_slot.alloc(c, sizeof(uint32_t) * nb);
    zero(c, kp.blk_slot.get(), kp.blk_slot.size());
    kp.choice_stats.alloc(c, sizeof(unsigned long long) * 3);
    zero(c, kp.choice_stats.get(), kp.choice_stats.size());
    kp.own_code = true;
    kp.mp.blk_slot = kp.blk_slot.as<uint32_t>();
    kp.dev_code.alloc(c, sizeof(Instr) * (size_t)std::min<uint32_t>(kPlanSlots, next_pow2(std::max<uint32_t>(2 * nl, 16))) *
                             kp.mp.plan_len);
    HB_HIP(hipMemcpyAsync(kp.dev_code.get(), kp.code.data(), sizeof(Instr) * kp.code.size(), hipMemcpyHostToDevice,
                          c->stream));
    kp.mp.plan = kp.dev_code.as<Instr>();
    if (nl == 0) return;
    DevBuf feat;
    LearnParams L;
    block_features(c, kp, R, feat, L, part.big.as<uint32_t>(), nl);
    DevBuf y(c, sizeof(float) * 2 * (size_t)nl * ns);
    c->host_timed("predict", [&] { model_forward(c, c->model, feat.as<float>(), (uint64_t)nl * ns, y.as<float>()); });

    C.y = y.as<float>();
    C.blocks = part.big.as<uint32_t>();
    C.blk_size = kp.mp.blk_size;
    C.n_blocks = nl;
    C.n_spec = ns;
    C.n_rules = n_rules;
    C.n_slots = std::min<uint32_t>(kPlanSlots, next_pow2(std::max<uint32_t>(2 * nl, 16)));
    C.plan_len = kp.mp.plan_len;
    C.rows = kp.mp.rows == 64 ? 64u : kp.mp.rows == 32 ? 32u : 16u;
    C.sparse_rows = kp.mp.sparse_rows;
    for (uint32_t x = 0; x < ns; ++x) C.spec_kind[x] = (uint8_t)R.specs[x].op;
    DevBuf keys(c, sizeof(unsigned long long) * C.n_slots);
    zero(c, keys.get(), keys.size());
    C.keys = keys.as<unsigned long long>();
    C.code = kp.dev_code.as<Instr>();
    C.blk_slot = kp.blk_slot.as<uint32_t>();
    C.stats = kp.choice_stats.as<unsigned long long>();
    kp.choice_cost.alloc(c, 2 * sizeof(float));
    zero(c, kp.choice_cost.get(), kp.choice_cost.size());
    C.cost = kp.choice_cost.as<float>();
    c->timed("plan_choice", [&] { return launch_plan_choice(C, c->stream); });
    kp.cost_pending = true;
}

void settle_learned(Ctx* c, std::vector<KeyPlan>& kps) {
    bool any = false;
    for (KeyPlan& kp : kps)
        if (kp.cost_pending) {
            HB_HIP(hipMemcpyAsync(kp.predicted, kp.choice_cost.get(), sizeof(kp.predicted), hipMemcpyDeviceToHost,
                                  c->stream));
            any = true;
        }
    if (!any) return;
    c->sync();
    // per-block plans are kept only when the model expects them to save at
    // least the context's minimum (a quarter by default) of the partition's
    // cost; otherwise every block runs the heuristic plan (slot 0).  Each
    // distinct plan is fetched through the scalar cache, which one shared
    // plan does not miss, and predicted savings of 11-20% on the two-key
    // recipes measured 1-3% slower kernels
    for (KeyPlan& kp : kps) {
        if (!kp.cost_pending) continue;
        kp.cost_pending = false;
        const float* pc = kp.predicted;
        if (c->learned_min_saving > 0.f && !(pc[1] < (1.f - c->learned_min_saving) * pc[0])) {
            kp.mp.blk_slot = nullptr;
            kp.discarded = true;
        }
    }
}

static void log_collect(Ctx* c, uint32_t rel_id, uint32_t rs_id, uint32_t samples, uint64_t seed, float* features,
                        float* labels, uint32_t* meta, uint64_t* counts, uint64_t cap, uint64_t* n_rows) {
    Relation& rel = get_rel(c, rel_id);
    RuleSet& rs = get_rs(c, rs_id, rel_id);
    if (!n_rows) fail(HB_ERR_INVALID_ARG, "NULL n_rows");
    if (samples == 0 || samples > 4096) fail(HB_ERR_INVALID_ARG, "samples must be in [1, 4096]");
    if (!rs.partitioned) fail(HB_ERR_STATE, "hb_partition must run before hb_log_collect");
    if (rs.ordered) fail(HB_ERR_INVALID_ARG, "cost-model logs take rule sets of t.A = s.A and t.A ~ s.A predicates only");
    uint64_t total = 0;
    struct Part {
        std::vector<float> f;
        std::vector<unsigned long long> cnt;
        std::vector<uint16_t> pred;
        uint32_t nb = 0, ns = 0;
    };
    std::vector<Part> parts(rs.keys.size());
    for (size_t ka = 0; ka < rs.keys.size(); ++ka) {
        if (rel.parts.at(rs.keys[ka]).n_tiles == 0) continue;
        KeyPlan kp;
        KeyRes R;
        if (!prepare_key(c, rel, rs, ka, kp, R, false)) continue;
        DevBuf feat;
        LearnParams L;
        block_features(c, kp, R, feat, L, nullptr, 0);
        const size_t rows = (size_t)kp.mp.n_blocks * L.n_spec;
        DevBuf cnt(c, sizeof(unsigned long long) * 4 * std::max<size_t>(rows, 1));
        zero(c, cnt.get(), cnt.size());
        L.counts = cnt.as<unsigned long long>();
        L.samples = samples;
        L.seed = seed ^ ((uint64_t)ka << 56);
        c->timed("log", [&] { return launch_log_samples(L, c->stream); });
        Part& pt = parts[ka];
        pt.nb = kp.mp.n_blocks;
        pt.ns = L.n_spec;
        pt.f.resize(rows * kFeatures);
        pt.cnt.resize(rows * 4);
        for (uint32_t x = 0; x < L.n_spec; ++x) pt.pred.push_back(L.spec[x].pred);
        if (rows) {
            HB_HIP(hipMemcpyAsync(pt.f.data(), feat.get(), sizeof(float) * pt.f.size(), hipMemcpyDeviceToHost, c->stream));
            HB_HIP(hipMemcpyAsync(pt.cnt.data(), cnt.get(), sizeof(unsigned long long) * pt.cnt.size(),
                                  hipMemcpyDeviceToHost, c->stream));
        }
        c->sync();
        total += rows;
    }
    *n_rows = total;
    if (cap < total) fail(HB_ERR_CAPACITY, "row capacity " + std::to_string(cap) + " < " + std::to_string(total));
    uint64_t o = 0;
    for (size_t ka = 0; ka < parts.size(); ++ka) {
        const Part& pt = parts[ka];
        for (uint32_t b = 0; b < pt.nb; ++b)
            for (uint32_t x = 0; x < pt.ns; ++x, ++o) {
                const size_t r = (size_t)b * pt.ns + x;
                if (features) std::memcpy(features + o * kFeatures, pt.f.data() + r * kFeatures, sizeof(float) * kFeatures);
                const double lanes = (double)pt.cnt[r * 4 + 0], first = (double)pt.cnt[r * 4 + 3];
                const double cyc = (double)pt.cnt[r * 4 + 2];
                if (labels) {
                    labels[o * 2 + 0] = (float)(lanes > 0 ? first / lanes : 0.0);
                    labels[o * 2 + 1] = (float)(std::log2(1.0 + (lanes > 0 ? cyc / (lanes / 64.0) : 0.0)) / 16.0);
                }
                if (meta) {
                    meta[o * 3 + 0] = (uint32_t)ka;
                    meta[o * 3 + 1] = b;
                    meta[o * 3 + 2] = pt.pred[x];
                }
                if (counts)
                    for (int k = 0; k < 4; ++k) counts[o * 4 + k] = pt.cnt[r * 4 + k];
            }
    }
}

// Algorithmic cost model of pair evaluation (int32 lane-ops): a fixed part
// per evaluated lane plus a part per work unit (edit distance: text byte x
// 32-bit pattern word; Jaccard: merged list element; string equality: byte
// compared).  Value equality 2, |a-b| <= d 4, every exact filter 4 (a length
// or signature bound), string equality 2 + 1 per byte, Myers 17 per text
// byte and pattern word, the sorted merge 3 per element.
static const double kAlgBase[8] = {2, 4, 4, 4, 4, 2, 0, 0};
static const double kAlgUnit[8] = {0, 0, 0, 0, 0, 1, 17, 3};
// What the kernel issues per evaluated lane for the same operations (its
// signature filters take about 12 int32 operations: popcounts, a 24-bit
// multiply-add and the compare; the rest as above).
static const double kIssBase[8] = {1, 4, 3, 12, 12, 2, 4, 4};
static const double kIssUnit[8] = {0, 0, 0, 0, 0, 1, 17, 3};

// Seed of the random-order strategies: the rule set's predicate ids mixed
// together (fixed per rule set, so repeated calls evaluate identically).
static uint64_t strategy_seed(const std::vector<std::vector<uint32_t>>& rules) {
    uint64_t h = 0x48425053ull;
    for (const auto& r : rules)
        for (uint32_t p : r) h = h * 0x100000001B3ull + p + 1;
    return h;
}

static std::vector<PathRule> strategy_path(const std::vector<double>& sp, const std::vector<double>& cost,
                                           const std::vector<std::vector<uint32_t>>& rules, int plan) {
    switch (plan) {
    case HB_PLAN_GIVEN: return given_path(rules);
    case HB_PLAN_CHEAPEST: return epg_path(sp, cost, rules, Rank::kCheapest);
    case HB_PLAN_SELECTIVE: return epg_path(sp, cost, rules, Rank::kMostSelective);
    case HB_PLAN_RANDOM_PREDS: return shuffled_path(epg_path(sp, cost, rules), true, false, strategy_seed(rules));
    case HB_PLAN_RANDOM_RULES: return shuffled_path(epg_path(sp, cost, rules), false, true, strategy_seed(rules));
    default: return epg_path(sp, cost, rules);   // heuristic; the learned plan starts from it
    }
}

std::vector<PathRule> plan_path(const RuleSet& rs, int plan) { return strategy_path(rs.sp, rs.cost, rs.rules, plan); }

bool valid_plan(int plan) { return plan >= HB_PLAN_GIVEN && plan <= HB_PLAN_RANDOM_RULES; }

bool key_plan(Ctx* c, Relation& rel, RuleSet& rs, int plan, const std::vector<PathRule>& path, size_t ka,
              KeyPlan& kp, bool count, uint64_t* n_fallback) {
    if (plan != HB_PLAN_LEARNED) return build_key_plan(c, rel, rs, plan, path, ka, kp, count);
    KeyRes R;
    if (!prepare_key(c, rel, rs, ka, kp, R, count)) return false;
    c->host_timed("learned_plan", [&] { learned_key_plan(c, rel, rs, ka, kp, R, path, n_fallback); });
    return true;
}

void sort_pairs(Ctx* c, DevBuf& pairs, uint64_t n, uint64_t n_rows, DevBuf& result) {
    // packed pairs: j bits, then i bits
    const int nb = bit_width(n_rows > 1 ? n_rows - 1 : 1);
    std::vector<int> sh = shifts_for_bits(nb, 0);
    std::vector<int> shi = shifts_for_bits(nb, 32);
    sh.insert(sh.end(), shi.begin(), shi.end());
    result.alloc(c, sizeof(uint64_t) * std::max<uint64_t>(n, 1));
    if (n > 1) {
        if (n >= 0xFFFFFFFFull) fail(HB_ERR_LIMIT, "more than 2^32 matched pairs");
        DevBuf alt(c, sizeof(uint64_t) * n);
        DevBuf rtmp(c, radix_tmp_bytes((uint32_t)n));
        bool in_alt = false;
        c->timed("output_sort", [&] {
            return radix_sort_pairs(pairs.as<uint64_t>(), nullptr, alt.as<uint64_t>(), nullptr, (uint32_t)n, sh.data(),
                                    (int)sh.size(), rtmp.get(), &in_alt, c->stream);
        }, 24.0 * (double)n * (double)sh.size());
        HB_HIP(hipMemcpyAsync(result.get(), in_alt ? alt.get() : pairs.get(), sizeof(uint64_t) * n,
                              hipMemcpyDeviceToDevice, c->stream));
    } else if (n == 1) {
        HB_HIP(hipMemcpyAsync(result.get(), pairs.get(), 8, hipMemcpyDeviceToDevice, c->stream));
    }
}

static void run_match(Ctx* c, Relation& rel, RuleSet& rs, int plan, hb_work_stats* ws = nullptr) {
    if (rs.ordered && (ws || plan == HB_PLAN_LEARNED))
        fail(HB_ERR_INVALID_ARG, "learned plans and work counts take rule sets of t.A = s.A and t.A ~ s.A predicates only");
    const std::vector<PathRule> path = plan_path(rs, plan);
    std::vector<KeyPlan> kps;
    size_t total_code = 0;
    uint64_t n_learned = 0, n_fallback = 0, n_plans = 0;
    double pred_h = 0.0, pred_c = 0.0;
    for (size_t ka = 0; ka < rs.keys.size(); ++ka) {
        if (rel.parts.at(rs.keys[ka]).n_tiles == 0) continue;
        KeyPlan kp;
        if (!key_plan(c, rel, rs, plan, path, ka, kp, ws != nullptr, &n_fallback)) continue;
        if (!kp.own_code) total_code += kp.code.size();
        kps.push_back(std::move(kp));
    }
    settle_learned(c, kps);
    DevBuf code(c, sizeof(Instr) * std::max<size_t>(total_code, 1));
    DevBuf counts(c, sizeof(unsigned long long) * kCountSlots);
    if (ws) zero(c, counts.get(), counts.size());
    {
        std::vector<Instr> all;
        for (KeyPlan& kp : kps)
            if (!kp.own_code) all.insert(all.end(), kp.code.begin(), kp.code.end());
        if (!all.empty())
            HB_HIP(hipMemcpyAsync(code.get(), all.data(), sizeof(Instr) * all.size(), hipMemcpyHostToDevice, c->stream));
        size_t o = 0;
        for (KeyPlan& kp : kps) {
            kp.mp.counts = ws ? counts.as<unsigned long long>() : nullptr;
            if (kp.own_code) continue;
            kp.mp.plan = code.as<Instr>() + o;
            o += kp.code.size();
        }
    }
    DevBuf counter(c, 8);
    uint64_t cap = std::max<uint64_t>(1u << 20, rel.n_rows);
    DevBuf out(c, sizeof(uint64_t) * cap);
    uint64_t found = 0;
    uint64_t tiles = 0, launches = 0;
    for (int attempt = 0; attempt < 2; ++attempt) {
        zero(c, counter.get(), 8);
        tiles = launches = 0;
        for (KeyPlan& kp : kps) {
            kp.mp.out = out.as<uint64_t>();
            kp.mp.cap = cap;
            kp.mp.counter = counter.as<unsigned long long>();
            c->timed("match", [&] { return launch_match(kp.mp, c->stream); }, kp.feat_bytes);
            tiles += kp.mp.n_tiles;
            ++launches;
        }
        found = read1(c, counter.as<unsigned long long>());
        if (attempt == 0)
            for (KeyPlan& kp : kps) {
                if (!kp.own_code) continue;
                pred_h += kp.predicted[0];
                pred_c += kp.predicted[1];
                if (kp.discarded) {
                    n_fallback += kp.mp.n_blocks;
                    continue;
                }
                unsigned long long st[3];
                HB_HIP(hipMemcpyAsync(st, kp.choice_stats.get(), sizeof(st), hipMemcpyDeviceToHost, c->stream));
                c->sync();
                n_learned += st[0];
                n_fallback += kp.mp.n_blocks - st[0];
                n_plans += st[2];
            }
        if (ws || found <= cap) break;
        cap = found;
        out.alloc(c, sizeof(uint64_t) * cap);
    }
    if (ws) {
        std::vector<unsigned long long> h(counts.size() / sizeof(unsigned long long));
        HB_HIP(hipMemcpyAsync(h.data(), counts.get(), counts.size(), hipMemcpyDeviceToHost, c->stream));
        c->sync();
        std::memset(ws, 0, sizeof(*ws));
        for (int op = 0; op < HB_N_OPKINDS; ++op) {
            ws->waves[op] = h[op * 4 + 0];
            ws->lanes[op] = h[op * 4 + 1];
            ws->passed[op] = h[op * 4 + 2];
            ws->work[op] = h[op * 4 + 3];
        }
        ws->pairs = h[kCountPairs];
        double ops = 0.0, iss = 0.0, bops = 0.0;
        for (int op = 0; op < HB_N_OPKINDS; ++op) {
            const double units = op <= OP_JACF ? 0.0 : (double)ws->work[op];   // filters: no work units
            ops += kAlgBase[op] * ws->lanes[op] + kAlgUnit[op] * units;
            iss += kIssBase[op] * ws->lanes[op] + kIssUnit[op] * units;
            // cheap steps run for every lane of every row of the batch, or
            // for every lane once per round of the per-lane form; exact ones
            // per pair
            bops += op <= OP_JACF ? kIssBase[op] * ((double)ws->waves[op] * c->rows_per_wave + (double)ws->work[op]) * 64
                                  : kIssBase[op] * ws->lanes[op] + kIssUnit[op] * ws->work[op];
        }
        ws->lane_ops = ops;
        ws->issued_ops = iss;
        ws->batch_ops = bops;
        ws->matched = found;
        ws->launches = launches;
        return;
    }
    sort_pairs(c, out, found, rel.n_rows, rs.result);
    rs.n_result = found;
    rs.has_result = true;
    rs.result_plan = plan;
    c->last.candidate_pairs = rs.candidates;
    c->last.matched_pairs = found;
    c->last.tiles = tiles;
    c->last.launches = launches;
    c->last.learned_blocks = n_learned;
    c->last.fallback_blocks = n_fallback;
    c->last.learned_plans = n_plans;
    c->last.predicted_heuristic = pred_h;
    c->last.predicted_chosen = pred_c;
}

static void match_work(Ctx* c, uint32_t rel_id, uint32_t rs_id, int plan, hb_work_stats* ws) {
    Relation& rel = get_rel(c, rel_id);
    RuleSet& rs = get_rs(c, rs_id, rel_id);
    if (!ws) fail(HB_ERR_INVALID_ARG, "NULL stats");
    if (!valid_plan(plan)) fail(HB_ERR_INVALID_ARG, "unknown plan");
    if (!rs.partitioned) fail(HB_ERR_STATE, "hb_partition must run before hb_match_work");
    run_match(c, rel, rs, plan, ws);
}

static void match(Ctx* c, uint32_t rel_id, uint32_t rs_id, int plan, uint64_t* out, int out_on_device, uint64_t cap,
                  uint64_t* n_pairs) {
    Relation& rel = get_rel(c, rel_id);
    RuleSet& rs = get_rs(c, rs_id, rel_id);
    if (!n_pairs) fail(HB_ERR_INVALID_ARG, "NULL n_pairs");
    if (!valid_plan(plan)) fail(HB_ERR_INVALID_ARG, "unknown plan");
    if (!rs.partitioned) fail(HB_ERR_STATE, "hb_partition must run before hb_match");
    if (!(rs.has_result && rs.result_plan == plan)) run_match(c, rel, rs, plan);
    *n_pairs = rs.n_result;
    if (cap < rs.n_result) fail(HB_ERR_CAPACITY, "output capacity " + std::to_string(cap) + " < " + std::to_string(rs.n_result));
    if (rs.n_result) {
        if (!out) fail(HB_ERR_INVALID_ARG, "NULL output buffer");
        HB_HIP(hipMemcpyAsync(out, rs.result.get(), sizeof(uint64_t) * rs.n_result,
                              out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
    }
    c->sync();
}

// hb_match without allocation: the same plans (all but the learned one,
// whose per-block plans need buffers of their own), kernels and sort, with
// every device buffer of the call carved in turn from the device's scratch
// array, and the sorted pairs written to the caller's device buffer.  The
// indexes a match reads (q-gram indexes, character signatures) are built by
// hb_compile_rules, so nothing is cached here.
static void match_noalloc(Ctx* c, uint32_t rel_id, uint32_t rs_id, int plan, uint64_t* out, uint64_t cap,
                          uint64_t* n_pairs) {
    Relation& rel = get_rel(c, rel_id);
    RuleSet& rs = get_rs(c, rs_id, rel_id);
    if (!n_pairs) fail(HB_ERR_INVALID_ARG, "NULL n_pairs");
    if (!valid_plan(plan)) fail(HB_ERR_INVALID_ARG, "unknown plan");
    if (plan == HB_PLAN_LEARNED) fail(HB_ERR_INVALID_ARG, "hb_match_noalloc takes every plan but the learned one");
    if (!rs.partitioned) fail(HB_ERR_STATE, "hb_partition must run before hb_match_noalloc");
    if (!c->scratch) fail(HB_ERR_HIP, "no scratch array on this device: " + c->scratch_err);
    *n_pairs = 0;
    struct ArenaScope {
        Ctx* c;
        ArenaScope(Ctx* cc, uint8_t* base, size_t bytes) : c(cc) {
            c->arena = base;
            c->arena_cap = bytes;
            c->arena_used = 0;
        }
        ~ArenaScope() {
            c->arena = nullptr;
            c->arena_cap = c->arena_used = 0;
        }
    } scope(c, c->scratch, (size_t)HB_NOALLOC_SCRATCH_BYTES);

    const std::vector<PathRule> path = plan_path(rs, plan);
    std::vector<KeyPlan> kps;
    size_t total_code = 0;
    for (size_t ka = 0; ka < rs.keys.size(); ++ka) {
        if (rel.parts.at(rs.keys[ka]).n_tiles == 0) continue;
        KeyPlan kp;
        if (!build_key_plan(c, rel, rs, plan, path, ka, kp, false)) continue;
        total_code += kp.code.size();
        kps.push_back(std::move(kp));
    }
    DevBuf counter(c, 8);
    zero(c, counter.get(), 8);   // the array keeps the previous call's contents
    DevBuf code(c, sizeof(Instr) * std::max<size_t>(total_code, 1));
    std::vector<Instr> all;
    for (KeyPlan& kp : kps) all.insert(all.end(), kp.code.begin(), kp.code.end());
    if (!all.empty())
        HB_HIP(hipMemcpyAsync(code.get(), all.data(), sizeof(Instr) * all.size(), hipMemcpyHostToDevice, c->stream));
    // the rest of the array: unsorted pairs, then the sort's histograms
    const size_t left = c->arena_cap - std::min(c->arena_cap, ((c->arena_used + 255) & ~(size_t)255) + 512);
    uint64_t cap_s = std::min<uint64_t>(left / 8, 0xFFFFFFFEull);
    while (cap_s > 0 && cap_s * 8 + radix_tmp_bytes((uint32_t)cap_s) > left) cap_s -= std::max<uint64_t>(cap_s / 64, 1);
    DevBuf unsorted(c, sizeof(uint64_t) * std::max<uint64_t>(cap_s, 1));
    size_t o = 0;
    for (KeyPlan& kp : kps) {
        kp.mp.counts = nullptr;
        kp.mp.plan = code.as<Instr>() + o;
        o += kp.code.size();
        kp.mp.out = unsorted.as<uint64_t>();
        kp.mp.cap = cap_s;
        kp.mp.counter = counter.as<unsigned long long>();
        HB_HIP(launch_match(kp.mp, c->stream));
    }
    const uint64_t found = read1(c, counter.as<unsigned long long>());
    *n_pairs = found;
    if (cap < found) fail(HB_ERR_CAPACITY, "output capacity " + std::to_string(cap) + " < " + std::to_string(found));
    if (cap_s < found)
        fail(HB_ERR_LIMIT, "the scratch array holds " + std::to_string(cap_s) + " unsorted pairs, the call found " +
                               std::to_string(found));
    if (found && !out) fail(HB_ERR_INVALID_ARG, "NULL output buffer");
    if (found > 1) {
        // the caller's buffer is the sort's second buffer
        const int nb = bit_width(rel.n_rows > 1 ? rel.n_rows - 1 : 1);
        std::vector<int> sh = shifts_for_bits(nb, 0);
        std::vector<int> shi = shifts_for_bits(nb, 32);
        sh.insert(sh.end(), shi.begin(), shi.end());
        DevBuf rtmp(c, radix_tmp_bytes((uint32_t)found));
        bool in_alt = false;
        HB_HIP(radix_sort_pairs(unsorted.as<uint64_t>(), nullptr, out, nullptr, (uint32_t)found, sh.data(),
                                (int)sh.size(), rtmp.get(), &in_alt, c->stream));
        if (!in_alt)
            HB_HIP(hipMemcpyAsync(out, unsorted.get(), sizeof(uint64_t) * found, hipMemcpyDeviceToDevice, c->stream));
    } else if (found == 1) {
        HB_HIP(hipMemcpyAsync(out, unsorted.get(), 8, hipMemcpyDeviceToDevice, c->stream));
    }
    c->sync();
}

}  // namespace hb

// ============================================================ C ABI

using hb::Ctx;
using hb::Failure;


extern "C" {

const char* hb_version(void) { return "hb 0.1 (gfx950)"; }

hb_status hb_create(hb_ctx** out, int device, hb_alloc_fn alloc, hb_free_fn free_fn, void* user, void* stream) {
    if (!out) return HB_ERR_INVALID_ARG;
    *out = nullptr;
    if ((alloc == nullptr) != (free_fn == nullptr)) return HB_ERR_INVALID_ARG;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return HB_ERR_HIP;
    if (hipSetDevice(device) != hipSuccess) return HB_ERR_HIP;
    hb_ctx* h = new (std::nothrow) hb_ctx();
    if (!h) return HB_ERR_OOM;
    h->c.device = device;
    h->c.alloc_fn = alloc;
    h->c.free_fn = free_fn;
    h->c.user = user;
    if (stream) {
        h->c.stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&h->c.stream, hipStreamNonBlocking) != hipSuccess) {
            delete h;
            return HB_ERR_HIP;
        }
        h->c.own_stream = true;
    }
    int lds = 65536;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess) lds = 65536;
    h->c.lds_limit = (uint32_t)lds;
    // this device's copy of the allocation-free entry point's scratch array
    h->c.scratch = hb::scratch_address(device, &h->c.scratch_err);
    *out = h;
    return HB_OK;
}

void hb_destroy(hb_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->c.device);
    if (ctx->c.copy_stream) (void)hipStreamSynchronize(ctx->c.copy_stream);
    (void)hipStreamSynchronize(ctx->c.stream);
    ctx->c.drain_profile();
    ctx->c.batches.clear();
    ctx->c.rulesets.clear();
    ctx->c.rels.clear();
    (void)hipStreamSynchronize(ctx->c.stream);
    if (ctx->c.copy_stream) (void)hipStreamDestroy(ctx->c.copy_stream);
    if (ctx->c.own_stream) (void)hipStreamDestroy(ctx->c.stream);
    delete ctx;
}

const char* hb_last_error(const hb_ctx* ctx) { return ctx ? ctx->c.err.c_str() : "NULL context"; }

hb_status hb_load_relation(hb_ctx* ctx, uint32_t n_rows, uint32_t n_cols, const hb_column* cols, int on_device,
                           uint32_t* rel_id) {
    return guard(ctx, [&](Ctx* c) { hb::load_relation(c, n_rows, n_cols, cols, on_device, rel_id); });
}

hb_status hb_load_relation_async(hb_ctx* ctx, uint32_t n_rows, uint32_t n_cols, const hb_column* cols,
                                 int on_device, uint32_t* rel_id) {
    return guard(ctx, [&](Ctx* c) { hb::load_relation_async(c, n_rows, n_cols, cols, on_device, rel_id); });
}

hb_status hb_release_relation(hb_ctx* ctx, uint32_t rel_id) {
    return guard(ctx, [&](Ctx* c) {
        auto r = c->rels.find(rel_id);
        if (r == c->rels.end()) hb::fail(HB_ERR_STALE_ID, "unknown relation id " + std::to_string(rel_id));
        if (r->second->pending) HB_HIP(hipEventSynchronize(r->second->ready));   // its copies are done
        for (auto it = c->rulesets.begin(); it != c->rulesets.end();) {
            if (it->second->rel_id == rel_id) it = c->rulesets.erase(it); else ++it;
        }
        c->rels.erase(rel_id);
    });
}

hb_status hb_compile_rules(hb_ctx* ctx, uint32_t rel_id, uint32_t n_rules, const hb_rule* rules, uint32_t* ruleset_id) {
    return guard(ctx, [&](Ctx* c) { hb::compile_rules(c, rel_id, n_rules, rules, ruleset_id); });
}

hb_status hb_partition(hb_ctx* ctx, uint32_t rel_id, uint32_t ruleset_id, uint64_t* n_candidate_pairs) {
    return guard(ctx, [&](Ctx* c) { hb::partition(c, rel_id, ruleset_id, n_candidate_pairs); });
}

hb_status hb_match(hb_ctx* ctx, uint32_t rel_id, uint32_t ruleset_id, int32_t plan, uint64_t* out_pairs,
                   int out_on_device, uint64_t capacity, uint64_t* n_pairs) {
    return guard(ctx, [&](Ctx* c) { hb::match(c, rel_id, ruleset_id, plan, out_pairs, out_on_device, capacity, n_pairs); });
}

hb_status hb_match_noalloc(hb_ctx* ctx, uint32_t rel_id, uint32_t ruleset_id, int32_t plan, uint64_t* out_pairs,
                           uint64_t capacity, uint64_t* n_pairs) {
    return guard(ctx, [&](Ctx* c) { hb::match_noalloc(c, rel_id, ruleset_id, plan, out_pairs, capacity, n_pairs); });
}

hb_status hb_set_rows_per_wave(hb_ctx* ctx, uint32_t rows) {
    return guard(ctx, [&](Ctx* c) {
        if (rows != 16 && rows != 32 && rows != 64) hb::fail(HB_ERR_INVALID_ARG, "rows per wave batch must be 16, 32 or 64");
        c->rows_per_wave = rows;
        for (auto& it : c->rulesets) it.second->has_result = false;   // a later hb_match evaluates again
    });
}

hb_status hb_set_learned_min_saving(hb_ctx* ctx, float min_saving) {
    return guard(ctx, [&](Ctx* c) {
        if (!(min_saving >= 0.f && min_saving < 1.f)) hb::fail(HB_ERR_INVALID_ARG, "the minimum saving must be in [0, 1)");
        c->learned_min_saving = min_saving;
        for (auto& it : c->rulesets) it.second->has_result = false;
    });
}

hb_status hb_costmodel_select(hb_ctx* ctx, int which) {
    return guard(ctx, [&](Ctx* c) {
        if (which != HB_MODEL_BLOCK && which != HB_MODEL_PAIR)
            hb::fail(HB_ERR_INVALID_ARG, "model must be HB_MODEL_BLOCK or HB_MODEL_PAIR");
        c->model_sel = which;
    });
}

hb_status hb_set_cost_estimate(hb_ctx* ctx, int source, uint32_t samples, uint64_t seed) {
    return guard(ctx, [&](Ctx* c) {
        if (source != HB_COST_STATIC && source != HB_COST_PAIR_NET)
            hb::fail(HB_ERR_INVALID_ARG, "source must be HB_COST_STATIC or HB_COST_PAIR_NET");
        if (samples == 0 || samples > hb::kMaxPairSamples) hb::fail(HB_ERR_INVALID_ARG, "samples must be in [1, 65536]");
        c->cost_source = source;
        c->cost_samples = samples;
        c->cost_seed = seed;
    });
}

hb_status hb_pair_log_collect(hb_ctx* ctx, uint32_t rel_id, uint32_t ruleset_id, uint32_t samples, uint64_t seed,
                              float* features, float* labels, uint32_t* pairs, uint64_t cap_rows, uint64_t* n_rows) {
    return guard(ctx, [&](Ctx* c) {
        hb::pair_log_collect(c, rel_id, ruleset_id, samples, seed, features, labels, pairs, cap_rows, n_rows);
    });
}

hb_status hb_set_pack_small_blocks(hb_ctx* ctx, int on) {
    return guard(ctx, [&](Ctx* c) { c->pack_small_blocks = on != 0; });
}

hb_status hb_set_sparse_rows(hb_ctx* ctx, uint32_t max_rows) {
    return guard(ctx, [&](Ctx* c) {
        if (max_rows > (uint32_t)hb::kMaxSparseRows) hb::fail(HB_ERR_INVALID_ARG, "the per-lane threshold must be at most 32");
        c->sparse_rows = max_rows;
        for (auto& it : c->rulesets) it.second->has_result = false;
    });
}

hb_status hb_match_work(hb_ctx* ctx, uint32_t rel_id, uint32_t ruleset_id, int32_t plan, hb_work_stats* out) {
    return guard(ctx, [&](Ctx* c) { hb::match_work(c, rel_id, ruleset_id, plan, out); });
}

hb_status hb_log_collect(hb_ctx* ctx, uint32_t rel_id, uint32_t ruleset_id, uint32_t samples, uint64_t seed,
                         float* features, float* labels, uint32_t* meta, uint64_t* counts, uint64_t cap_rows,
                         uint64_t* n_rows) {
    return guard(ctx, [&](Ctx* c) {
        hb::log_collect(c, rel_id, ruleset_id, samples, seed, features, labels, meta, counts, cap_rows, n_rows);
    });
}

hb_status hb_ruleset_estimates(hb_ctx* ctx, uint32_t ruleset_id, double* sp, double* cost, uint32_t cap, uint32_t* n) {
    return guard(ctx, [&](Ctx* c) {
        auto it = c->rulesets.find(ruleset_id);
        if (it == c->rulesets.end()) hb::fail(HB_ERR_STALE_ID, "unknown rule set id");
        const auto& rs = *it->second;
        if (!n) hb::fail(HB_ERR_INVALID_ARG, "NULL n");
        *n = (uint32_t)rs.distinct.size();
        for (uint32_t p = 0; p < rs.distinct.size() && p < cap; ++p) {
            if (sp) sp[p] = rs.sp[p];
            if (cost) cost[p] = rs.cost[p];
        }
    });
}

hb_status hb_ruleset_buckets(hb_ctx* ctx, uint32_t ruleset_id, uint32_t pred, uint64_t* counts, uint64_t* n_valid) {
    return guard(ctx, [&](Ctx* c) {
        auto it = c->rulesets.find(ruleset_id);
        if (it == c->rulesets.end()) hb::fail(HB_ERR_STALE_ID, "unknown rule set id");
        const auto& rs = *it->second;
        if (pred >= rs.distinct.size()) hb::fail(HB_ERR_INVALID_ARG, "predicate index out of range");
        if (counts) std::memcpy(counts, rs.buckets[pred].data(), sizeof(uint64_t) * hb::kLshK);
        if (n_valid) *n_valid = rs.bucket_n[pred];
    });
}

hb_status hb_epg_path(uint32_t n_preds, const double* sp, const double* cost, uint32_t n_rules,
                      const uint32_t* rule_len, const uint32_t* rule_preds, uint32_t* out_rules, uint32_t* out_preds,
                      uint32_t* out_len) {
    return hb_plan_path(HB_PLAN_HEURISTIC, n_preds, sp, cost, n_rules, rule_len, rule_preds, out_rules, out_preds,
                        out_len);
}

hb_status hb_plan_path(uint32_t plan, uint32_t n_preds, const double* sp, const double* cost, uint32_t n_rules,
                       const uint32_t* rule_len, const uint32_t* rule_preds, uint32_t* out_rules, uint32_t* out_preds,
                       uint32_t* out_len) {
    if (!sp || !cost || !rule_len || !rule_preds || !out_rules || !out_preds || !out_len) return HB_ERR_INVALID_ARG;
    if (!hb::valid_plan((int)plan) || plan == HB_PLAN_LEARNED) return HB_ERR_INVALID_ARG;
    for (uint32_t p = 0; p < n_preds; ++p)
        if (!(cost[p] > 0.0) || !(sp[p] >= 0.0 && sp[p] <= 1.0)) return HB_ERR_INVALID_ARG;
    try {
        std::vector<std::vector<uint32_t>> rules(n_rules);
        size_t o = 0;
        for (uint32_t r = 0; r < n_rules; ++r) {
            for (uint32_t x = 0; x < rule_len[r]; ++x) {
                uint32_t p = rule_preds[o++];
                if (p >= n_preds) return HB_ERR_INVALID_ARG;
                rules[r].push_back(p);
            }
        }
        std::vector<double> vsp(sp, sp + n_preds), vc(cost, cost + n_preds);
        auto path = hb::strategy_path(vsp, vc, rules, (int)plan);
        uint32_t w = 0;
        for (uint32_t r = 0; r < path.size(); ++r) {
            out_rules[r] = path[r].rule;
            for (uint32_t p : path[r].preds) out_preds[w++] = p;
        }
        *out_len = w;
        return HB_OK;
    } catch (...) {
        return HB_ERR_OOM;
    }
}

hb_status hb_costmodel_init(hb_ctx* ctx, uint64_t seed) {
    return guard(ctx, [&](Ctx* c) { hb::costmodel_init(c, seed); });
}

hb_status hb_costmodel_set_params(hb_ctx* ctx, const float* params, uint32_t n) {
    return guard(ctx, [&](Ctx* c) { hb::costmodel_set(c, params, n); });
}

hb_status hb_costmodel_get_params(hb_ctx* ctx, float* params, uint32_t n) {
    return guard(ctx, [&](Ctx* c) { hb::costmodel_get(c, params, n); });
}

hb_status hb_costmodel_train(hb_ctx* ctx, const float* x, const float* t, uint64_t n_rows, int on_device,
                             uint32_t epochs, uint32_t batch, float lr, float* final_loss) {
    return guard(ctx, [&](Ctx* c) { hb::costmodel_train(c, x, t, n_rows, on_device, epochs, batch, lr, final_loss); });
}

hb_status hb_costmodel_predict(hb_ctx* ctx, const float* x, uint64_t n_rows, int on_device, float* y,
                               int y_on_device) {
    return guard(ctx, [&](Ctx* c) { hb::costmodel_predict(c, x, n_rows, on_device, y, y_on_device); });
}

hb_status hb_costmodel_trace(hb_ctx* ctx, const float* x, const float* t, uint32_t n_rows, float* out,
                             uint64_t out_len) {
    return guard(ctx, [&](Ctx* c) { hb::costmodel_trace(c, x, t, n_rows, out, out_len); });
}

hb_status hb_costmodel_adam_step(hb_ctx* ctx, const float* grads, float lr) {
    return guard(ctx, [&](Ctx* c) { hb::costmodel_adam(c, grads, lr); });
}

hb_status hb_costmodel_save(hb_ctx* ctx, const char* path) {
    return guard(ctx, [&](Ctx* c) { hb::costmodel_save(c, path); });
}

hb_status hb_costmodel_load(hb_ctx* ctx, const char* path) {
    return guard(ctx, [&](Ctx* c) { hb::costmodel_load(c, path); });
}

hb_status hb_profile_enable(hb_ctx* ctx, int on) {
    return guard(ctx, [&](Ctx* c) { c->profiling = on != 0; });
}

hb_status hb_profile_query(hb_ctx* ctx, const char* name, double* total_ms, uint64_t* launches) {
    return guard(ctx, [&](Ctx* c) {
        if (!name) hb::fail(HB_ERR_INVALID_ARG, "NULL name");
        c->drain_profile();
        auto it = c->prof.find(name);
        if (total_ms) *total_ms = it == c->prof.end() ? 0.0 : it->second.ms;
        if (launches) *launches = it == c->prof.end() ? 0 : it->second.launches;
    });
}

hb_status hb_profile_bytes(hb_ctx* ctx, const char* name, double* bytes) {
    return guard(ctx, [&](Ctx* c) {
        if (!name || !bytes) hb::fail(HB_ERR_INVALID_ARG, "NULL argument");
        c->drain_profile();
        auto it = c->prof.find(name);
        *bytes = it == c->prof.end() ? 0.0 : it->second.bytes;
    });
}

hb_status hb_profile_reset(hb_ctx* ctx) {
    return guard(ctx, [&](Ctx* c) {
        c->drain_profile();
        c->prof.clear();
    });
}

hb_status hb_last_match_stats(hb_ctx* ctx, hb_match_stats* out) {
    return guard(ctx, [&](Ctx* c) {
        if (!out) hb::fail(HB_ERR_INVALID_ARG, "NULL out");
        *out = c->last;
    });
}

}  // extern "C"
