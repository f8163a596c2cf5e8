// Batched matching: many (relation, rule set) jobs matched together over
// one queue of all their key partitions' tiles, heaviest partitions first.
// Launch forms: every partition's own launch spread over concurrent
// streams, one one-wave workgroup per 16-row batch of a tile over the whole
// queue, or a persistent work-stealing grid; the form (and the grid's grab size and occupancy) can
// be picked by timing them on the batch's first items, and the batch's
// device work can be captured in a HIP graph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <memory>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/hb.h"
#include "hb_abi.h"
#include "hb_ctx.h"
#include "hb_internal.h"
#include "hb_keyplan.h"

namespace hb {

struct Batch {
    int plan = HB_PLAN_HEURISTIC;
    uint32_t flags = 0;
    struct Job {
        uint32_t rel_id = 0, rs_id = 0;
        const Relation* rel = nullptr;
        const RuleSet* rs = nullptr;
        uint64_t n_rows = 0, cap = 0, n_result = 0;
        DevBuf out, result;
    };
    std::vector<Job> jobs;
    std::vector<KeyPlan> kps;         // in queue order (heaviest first)
    std::vector<uint32_t> kp_job;
    DevBuf code, mps, prefix, cursor, counters;
    std::vector<uint64_t> h_prefix;
    uint64_t total = 0;
    uint32_t n_parts = 0, lds_bytes = 0, grid = 0, grab = 1, occupancy = 1;
    int form = 0;                     // kFormStreams / kFormMulti / kFormPersistent
    hipStream_t side = nullptr;       // graph launches (capture needs a non-default stream)
    hipStream_t lanes[4] = {nullptr, nullptr, nullptr, nullptr};   // concurrent partition launches
    hipEvent_t ev_lane[4] = {nullptr, nullptr, nullptr, nullptr};
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t learned_blocks = 0, fallback_blocks = 0;
    double tune_ms[32] = {0};
    uint32_t n_tuned = 0;

    ~Batch() {
        for (int x = 0; x < 4; ++x) {
            if (ev_lane[x]) (void)hipEventDestroy(ev_lane[x]);
            if (lanes[x]) (void)hipStreamDestroy(lanes[x]);
        }
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (ev_out) (void)hipEventDestroy(ev_out);
        if (side) (void)hipStreamDestroy(side);
    }
};

constexpr int kFormStreams = 0, kFormMulti = 1, kFormPersistent = 2;

static Batch& get_batch(Ctx* c, uint32_t id) {
    auto it = c->batches.find(id);
    if (it == c->batches.end()) fail(HB_ERR_STALE_ID, "unknown batch id");
    return *it->second;
}

// Every job's relation and rule set must still be the ones the batch was
// built from (their device memory is read by the batch's launches).
static void check_alive(Ctx* c, const Batch& B) {
    for (const Batch::Job& j : B.jobs) {
        auto r = c->rels.find(j.rel_id);
        auto s = c->rulesets.find(j.rs_id);
        if (r == c->rels.end() || r->second.get() != j.rel || s == c->rulesets.end() || s->second.get() != j.rs)
            fail(HB_ERR_STALE_ID, "a relation or rule set of the batch was released");
    }
}

// The per-partition parameters with each job's output buffer, in queue order.
static void upload_params(Ctx* c, Batch& B) {
    std::vector<MatchParams> h(B.n_parts);
    for (uint32_t p = 0; p < B.n_parts; ++p) {
        Batch::Job& j = B.jobs[B.kp_job[p]];
        MatchParams m = B.kps[p].mp;
        m.out = j.out.as<uint64_t>();
        m.cap = j.cap;
        m.counter = B.counters.as<unsigned long long>() + B.kp_job[p];
        m.counts = nullptr;
        h[p] = m;
    }
    HB_HIP(hipMemcpyAsync(B.mps.get(), h.data(), sizeof(MatchParams) * h.size(), hipMemcpyHostToDevice, c->stream));
}

// The batch's device work on stream s, in launch form `form`.  Streams:
// partition p (queue order) runs its own k_match launch on lane p mod 4,
// after s's counter reset and before s continues.  Multi: one workgroup per
// queue item.  Persistent: `grid` workgroups taking `grab` items per atomic.
// `total` < B.total limits the queue to its first items (timing samples;
// every form then runs exactly those items).
static void enqueue(Batch& B, uint64_t total, int form, uint32_t grab, uint32_t grid, hipStream_t s) {
    HB_HIP(launch_fill_u64(B.counters.as<unsigned long long>(), B.jobs.size(), 0ull, s));
    if (form == kFormMulti) {
        HB_HIP(launch_match_multi(B.mps.as<MatchParams>(), B.prefix.as<uint64_t>(), B.n_parts, total, B.lds_bytes, s));
        return;
    }
    if (form == kFormPersistent) {
        HB_HIP(launch_fill_u64(B.cursor.as<unsigned long long>(), 1, 0ull, s));
        HB_HIP(launch_match_persistent(B.mps.as<MatchParams>(), B.prefix.as<uint64_t>(), B.n_parts, total,
                                       B.cursor.as<unsigned long long>(), grab, grid, B.lds_bytes, s));
        return;
    }
    HB_HIP(hipEventRecord(B.ev_in, s));
    for (int x = 0; x < 4; ++x) HB_HIP(hipStreamWaitEvent(B.lanes[x], B.ev_in, 0));
    for (uint32_t p = 0; p < B.n_parts && B.h_prefix[p] < total; ++p) {
        const Batch::Job& j = B.jobs[B.kp_job[p]];
        MatchParams m = B.kps[p].mp;
        m.out = j.out.as<uint64_t>();
        m.cap = j.cap;
        m.counter = B.counters.as<unsigned long long>() + B.kp_job[p];
        m.counts = nullptr;
        m.n_tiles = std::min<uint64_t>(m.n_tiles, total - B.h_prefix[p]);   // a sample ends inside p
        HB_HIP(launch_match(m, B.lanes[p % 4]));
    }
    for (int x = 0; x < 4; ++x) {
        HB_HIP(hipEventRecord(B.ev_lane[x], B.lanes[x]));
        HB_HIP(hipStreamWaitEvent(s, B.ev_lane[x], 0));
    }
}

// Times each launch form on the first items of the queue (the heaviest
// partitions) and keeps the fastest: concurrent per-partition launches, one
// workgroup per item, or the persistent grid at each (grab, occupancy).
static void autotune(Ctx* c, Batch& B, int max_occ, int n_cu) {
    struct Cand {
        int form;
        uint32_t grab, occ;
    };
    std::vector<Cand> cands{{kFormStreams, 0, 0}};
    if (B.total <= kMaxTiles) cands.push_back({kFormMulti, 0, 0});
    std::vector<uint32_t> occs;
    for (int o = 1; o <= max_occ; o *= 2) occs.push_back((uint32_t)o);
    if (occs.back() != (uint32_t)max_occ) occs.push_back((uint32_t)max_occ);
    for (uint32_t occ : occs)
        for (uint32_t g : {1u, 4u}) cands.push_back({kFormPersistent, g, occ});
    const uint64_t sample = std::min<uint64_t>(B.total, (uint64_t)n_cu * max_occ * 64);
    hipEvent_t a, b;
    HB_HIP(hipEventCreate(&a));
    HB_HIP(hipEventCreate(&b));
    double best = 1e300;
    B.n_tuned = 0;
    for (const Cand& cd : cands) {
        const uint32_t grid = (uint32_t)n_cu * std::max<uint32_t>(cd.occ, 1);
        enqueue(B, sample, cd.form, cd.grab, grid, c->stream);   // warm
        HB_HIP(hipEventRecord(a, c->stream));
        enqueue(B, sample, cd.form, cd.grab, grid, c->stream);
        HB_HIP(hipEventRecord(b, c->stream));
        HB_HIP(hipEventSynchronize(b));
        float ms = 0.f;
        HB_HIP(hipEventElapsedTime(&ms, a, b));
        if (B.n_tuned < 32) B.tune_ms[B.n_tuned++] = ms;
        if (ms < best) {
            best = ms;
            B.form = cd.form;
            B.grab = cd.grab;
            B.occupancy = std::max<uint32_t>(cd.occ, 1);
            B.grid = grid;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
}

static void capture(Ctx* c, Batch& B) {
    if (B.exec) (void)hipGraphExecDestroy(B.exec);
    if (B.graph) (void)hipGraphDestroy(B.graph);
    B.exec = nullptr;
    B.graph = nullptr;
    HB_HIP(hipStreamSynchronize(c->stream));
    HB_HIP(hipStreamBeginCapture(B.side, hipStreamCaptureModeThreadLocal));
    try {
        enqueue(B, B.total, B.form, B.grab, B.grid, B.side);
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(B.side, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    HB_HIP(hipStreamEndCapture(B.side, &B.graph));
    HB_HIP(hipGraphInstantiate(&B.exec, B.graph, nullptr, nullptr, 0));
}

static void batch_create(Ctx* c, const hb_job* jobs, uint32_t n_jobs, int plan, uint32_t flags, uint32_t* id) {
    if (!id || (!jobs && n_jobs)) fail(HB_ERR_INVALID_ARG, "NULL argument");
    if (n_jobs == 0 || n_jobs > HB_MAX_BATCH_JOBS) fail(HB_ERR_INVALID_ARG, "n_jobs must be in [1, HB_MAX_BATCH_JOBS]");
    if (!valid_plan(plan)) fail(HB_ERR_INVALID_ARG, "unknown plan");
    if (flags & ~(uint32_t)(HB_BATCH_GRAPH | HB_BATCH_AUTOTUNE | HB_BATCH_FORM_MASK))
        fail(HB_ERR_INVALID_ARG, "unknown batch flags");
    if ((flags & HB_BATCH_AUTOTUNE) && (flags & HB_BATCH_FORM_MASK))
        fail(HB_ERR_INVALID_ARG, "a forced launch form excludes autotuning");
    auto B = std::make_shared<Batch>();
    B->plan = plan;
    B->flags = flags;
    std::vector<KeyPlan> kps;
    std::vector<uint32_t> kp_job;
    for (uint32_t j = 0; j < n_jobs; ++j) {
        Relation& rel = get_rel(c, jobs[j].rel_id);
        RuleSet& rs = get_rs(c, jobs[j].ruleset_id, jobs[j].rel_id);
        if (!rs.partitioned) fail(HB_ERR_STATE, "hb_partition must run on every job before hb_batch_create");
        if (rs.ordered) fail(HB_ERR_INVALID_ARG, "batches take rule sets of t.A = s.A and t.A ~ s.A predicates only");
        Batch::Job job;
        job.rel_id = jobs[j].rel_id;
        job.rs_id = jobs[j].ruleset_id;
        job.rel = &rel;
        job.rs = &rs;
        job.n_rows = rel.n_rows;
        job.cap = std::max<uint64_t>(1u << 16, rel.n_rows);
        job.out.alloc(c, sizeof(uint64_t) * job.cap);
        const std::vector<PathRule> path = plan_path(rs, plan);
        c->host_timed("batch_plans", [&] {
            for (size_t ka = 0; ka < rs.keys.size(); ++ka) {
                if (rel.parts.at(rs.keys[ka]).n_tiles == 0) continue;
                KeyPlan kp;
                if (!key_plan(c, rel, rs, plan, path, ka, kp, false, &B->fallback_blocks)) continue;
                kps.push_back(std::move(kp));
                kp_job.push_back(j);
            }
        });
        B->jobs.push_back(std::move(job));
    }
    // queue order: heaviest partitions first (tiles x plan length)
    std::vector<size_t> ord(kps.size());
    std::iota(ord.begin(), ord.end(), 0);
    auto weight = [&](size_t x) { return (double)kps[x].mp.n_tiles * std::max<uint32_t>(kps[x].mp.plan_len, 1); };
    std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return weight(a) > weight(b); });
    for (size_t x : ord) {
        B->kps.push_back(std::move(kps[x]));
        B->kp_job.push_back(kp_job[x]);
    }
    B->n_parts = (uint32_t)B->kps.size();
    settle_learned(c, B->kps);   // one read-back for every learned partition
    // plans: the shared-code ones in one device buffer
    size_t total_code = 0;
    for (const KeyPlan& kp : B->kps)
        if (!kp.own_code) total_code += kp.code.size();
    B->code.alloc(c, sizeof(Instr) * std::max<size_t>(total_code, 1));
    {
        std::vector<Instr> all;
        for (const KeyPlan& kp : B->kps)
            if (!kp.own_code) all.insert(all.end(), kp.code.begin(), kp.code.end());
        if (!all.empty())
            HB_HIP(hipMemcpyAsync(B->code.get(), all.data(), sizeof(Instr) * all.size(), hipMemcpyHostToDevice,
                                  c->stream));
        size_t o = 0;
        for (KeyPlan& kp : B->kps) {
            if (kp.own_code) continue;
            kp.mp.plan = B->code.as<Instr>() + o;
            o += kp.code.size();
        }
    }
    B->h_prefix.assign(B->n_parts + 1, 0);
    for (uint32_t p = 0; p < B->n_parts; ++p) {
        B->h_prefix[p + 1] = B->h_prefix[p] + B->kps[p].mp.n_tiles;
        B->lds_bytes = std::max(B->lds_bytes, B->kps[p].mp.lds_bytes);
    }
    B->total = B->h_prefix[B->n_parts];
    B->mps.alloc(c, sizeof(MatchParams) * std::max<uint32_t>(B->n_parts, 1));
    B->prefix.alloc(c, sizeof(uint64_t) * (B->n_parts + 1));
    B->cursor.alloc(c, sizeof(unsigned long long));
    B->counters.alloc(c, sizeof(unsigned long long) * B->jobs.size());
    HB_HIP(hipMemcpyAsync(B->prefix.get(), B->h_prefix.data(), sizeof(uint64_t) * (B->n_parts + 1),
                          hipMemcpyHostToDevice, c->stream));
    upload_params(c, *B);
    // grid: every CU, at the occupancy the LDS footprint allows
    int n_cu = 0, occ = 1;
    HB_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, c->device));
    HB_HIP(match_persistent_occupancy(B->lds_bytes, &occ));
    occ = std::max(occ, 1);
    B->occupancy = (uint32_t)occ;
    B->grid = (uint32_t)(n_cu * occ);
    B->form = kFormStreams;
    B->grab = 0;
    HB_HIP(hipStreamCreateWithFlags(&B->side, hipStreamNonBlocking));
    HB_HIP(hipEventCreateWithFlags(&B->ev_in, hipEventDisableTiming));
    HB_HIP(hipEventCreateWithFlags(&B->ev_out, hipEventDisableTiming));
    for (int x = 0; x < 4; ++x) {
        HB_HIP(hipStreamCreateWithFlags(&B->lanes[x], hipStreamNonBlocking));
        HB_HIP(hipEventCreateWithFlags(&B->ev_lane[x], hipEventDisableTiming));
    }
    if (flags & HB_BATCH_FORM_MASK) {
        const uint32_t f = flags & HB_BATCH_FORM_MASK;
        B->form = f == HB_BATCH_FORM_MULTI ? kFormMulti : f == HB_BATCH_FORM_PERSISTENT ? kFormPersistent : kFormStreams;
        B->grab = 1;
        if (B->form == kFormMulti && B->total > kMaxTiles)
            fail(HB_ERR_LIMIT, "more than 2^30 - 8 tiles for the one-workgroup-per-batch form");
    } else if ((flags & HB_BATCH_AUTOTUNE) && B->total > 0) {
        autotune(c, *B, occ, n_cu);
        c->batch_tuned = true;
        c->tuned_form = B->form;
        c->tuned_grab = B->grab;
        c->tuned_occupancy = B->occupancy;
    } else if (c->batch_tuned) {
        B->form = c->tuned_form;
        B->grab = c->tuned_grab;
        B->occupancy = std::min<uint32_t>(c->tuned_occupancy, (uint32_t)occ);
        B->grid = (uint32_t)n_cu * B->occupancy;
        if (B->form == kFormMulti && B->total > kMaxTiles) B->form = kFormStreams;
    }
    if (flags & HB_BATCH_GRAPH) c->host_timed("batch_capture", [&] { capture(c, *B); });
    c->sync();
    const uint32_t bid = c->next_id++;
    c->batches[bid] = B;
    *id = bid;
}

static void batch_run(Ctx* c, uint32_t id, uint64_t* n_total) {
    Batch& B = get_batch(c, id);
    check_alive(c, B);
    std::vector<unsigned long long> cnt(B.jobs.size());
    for (int attempt = 0; attempt < 2; ++attempt) {
        c->timed("batch_match", [&] {
            if (B.exec) {
                // the side stream runs the graph between the context stream's work
                HB_HIP(hipEventRecord(B.ev_out, c->stream));
                HB_HIP(hipStreamWaitEvent(B.side, B.ev_out, 0));
                HB_HIP(hipGraphLaunch(B.exec, B.side));
                HB_HIP(hipEventRecord(B.ev_out, B.side));
                HB_HIP(hipStreamWaitEvent(c->stream, B.ev_out, 0));
            } else {
                enqueue(B, B.total, B.form, B.grab, B.grid, c->stream);
            }
            return hipSuccess;
        });
        HB_HIP(hipMemcpyAsync(cnt.data(), B.counters.get(), sizeof(unsigned long long) * cnt.size(),
                              hipMemcpyDeviceToHost, c->stream));
        c->sync();
        bool over = false;
        for (size_t j = 0; j < B.jobs.size(); ++j)
            if (cnt[j] > B.jobs[j].cap) {
                over = true;
                B.jobs[j].cap = cnt[j];
                B.jobs[j].out.alloc(c, sizeof(uint64_t) * cnt[j]);
            }
        if (!over) break;
        if (attempt == 1) fail(HB_ERR_STATE, "internal: batch output grew between identical runs");
        upload_params(c, B);
        if (B.exec) capture(c, B);   // per-partition launches hold the buffers in their arguments
    }
    uint64_t total = 0;
    for (size_t j = 0; j < B.jobs.size(); ++j) {
        Batch::Job& job = B.jobs[j];
        sort_pairs(c, job.out, cnt[j], job.n_rows, job.result);
        job.n_result = cnt[j];
        total += cnt[j];
    }
    c->sync();
    if (n_total) *n_total = total;
}

static void batch_result(Ctx* c, uint32_t id, uint32_t job, uint64_t* out, int out_on_device, uint64_t cap,
                         uint64_t* n_pairs) {
    Batch& B = get_batch(c, id);
    if (!n_pairs) fail(HB_ERR_INVALID_ARG, "NULL n_pairs");
    if (job >= B.jobs.size()) fail(HB_ERR_INVALID_ARG, "job index out of range");
    const Batch::Job& j = B.jobs[job];
    *n_pairs = j.n_result;
    if (cap < j.n_result) fail(HB_ERR_CAPACITY, "output capacity " + std::to_string(cap) + " < " + std::to_string(j.n_result));
    if (j.n_result) {
        if (!out) fail(HB_ERR_INVALID_ARG, "NULL output buffer");
        HB_HIP(hipMemcpyAsync(out, j.result.get(), sizeof(uint64_t) * j.n_result,
                              out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
    }
    c->sync();
}

static void batch_info(Ctx* c, uint32_t id, hb_batch_info* info) {
    Batch& B = get_batch(c, id);
    if (!info) fail(HB_ERR_INVALID_ARG, "NULL info");
    std::memset(info, 0, sizeof(*info));
    info->n_jobs = (uint32_t)B.jobs.size();
    info->n_partitions = B.n_parts;
    info->work_items = B.total;
    info->grid = B.grid;
    info->grab = B.grab;
    info->form = B.form;
    info->occupancy = B.occupancy;
    info->lds_bytes = B.lds_bytes;
    info->graph = B.exec != nullptr;
    info->n_tuned = B.n_tuned;
    for (uint32_t x = 0; x < B.n_tuned && x < 32; ++x) info->tune_ms[x] = B.tune_ms[x];
    info->fallback_blocks = B.fallback_blocks;
}

}  // namespace hb

// ============================================================ C ABI

extern "C" {

hb_status hb_batch_create(hb_ctx* ctx, const hb_job* jobs, uint32_t n_jobs, int32_t plan, uint32_t flags,
                          uint32_t* batch_id) {
    return guard(ctx, [&](hb::Ctx* c) { hb::batch_create(c, jobs, n_jobs, plan, flags, batch_id); });
}

hb_status hb_batch_run(hb_ctx* ctx, uint32_t batch_id, uint64_t* n_pairs_total) {
    return guard(ctx, [&](hb::Ctx* c) { hb::batch_run(c, batch_id, n_pairs_total); });
}

hb_status hb_batch_result(hb_ctx* ctx, uint32_t batch_id, uint32_t job, uint64_t* out_pairs, int out_on_device,
                          uint64_t capacity, uint64_t* n_pairs) {
    return guard(ctx, [&](hb::Ctx* c) { hb::batch_result(c, batch_id, job, out_pairs, out_on_device, capacity, n_pairs); });
}

hb_status hb_batch_info_get(hb_ctx* ctx, uint32_t batch_id, hb_batch_info* info) {
    return guard(ctx, [&](hb::Ctx* c) { hb::batch_info(c, batch_id, info); });
}

hb_status hb_batch_destroy(hb_ctx* ctx, uint32_t batch_id) {
    return guard(ctx, [&](hb::Ctx* c) {
        auto it = c->batches.find(batch_id);
        if (it == c->batches.end()) hb::fail(HB_ERR_STALE_ID, "unknown batch id");
        c->sync();
        c->batches.erase(it);
    });
}

}  // extern "C"
