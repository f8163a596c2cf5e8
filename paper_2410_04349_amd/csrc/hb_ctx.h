// Host-side state of libhb shared by the entry-point files: error
// handling, device buffers owned through the context's allocator, the
// context, relations, rule sets and the cost model.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <chrono>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/hb.h"
#include "hb_internal.h"

namespace hb {

struct Failure {
    hb_status st;
    std::string msg;
};

[[noreturn]] inline void fail(hb_status st, const std::string& msg) { throw Failure{st, msg}; }

#define HB_HIP(expr)                                                                               \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) ::hb::fail(HB_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

struct Ctx;

// Device buffer owned through the context's allocator.
class DevBuf {
public:
    DevBuf() = default;
    DevBuf(Ctx* c, size_t bytes) { alloc(c, bytes); }
    ~DevBuf() { release(); }
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept { swap(o); }
    DevBuf& operator=(DevBuf&& o) noexcept {
        release();
        swap(o);
        return *this;
    }
    void alloc(Ctx* c, size_t bytes);
    void release();
    template <typename T>
    T* as() const { return static_cast<T*>(p_); }
    void* get() const { return p_; }
    size_t size() const { return n_; }

private:
    void swap(DevBuf& o) {
        std::swap(c_, o.c_);
        std::swap(p_, o.p_);
        std::swap(n_, o.n_);
        std::swap(borrowed_, o.borrowed_);
    }
    Ctx* c_ = nullptr;
    void* p_ = nullptr;
    size_t n_ = 0;
    bool borrowed_ = false;   // carved from the context's arena: never freed
};

struct Column {
    int32_t type = 0;
    uint32_t max_len = 0;
    double mean_len = 0.0;
    DevBuf off, bytes, values, valid;
};

struct GramIndex {
    uint32_t attr = 0, q = 0, max_cnt = 0, sig_words = 1;
    DevBuf off, cnt, codes, flags, sig;
    GramDev dev() const {
        GramDev g{};
        g.off = off.as<uint64_t>();
        g.cnt = cnt.as<uint32_t>();
        g.codes = codes.as<uint32_t>();
        g.flags = flags.as<uint8_t>();
        g.q = q;
        g.max_cnt = max_cnt;
        g.attr = attr;
        g.sig_words = sig_words;
        return g;
    }
};

struct Partition {
    uint32_t attr = 0, n_valid = 0, n_blocks = 0;
    uint64_t n_tiles = 0, pairs = 0;
    DevBuf perm, blk_start, blk_size, tile_prefix;
    DevBuf tile_blk;      // unit of each tile
    DevBuf big;           // blocks of >= kTile tuples (the ones with per-block plans)
    uint32_t n_big = 0;
    // windows of small blocks (MatchParams::unit_*); empty: units are blocks
    DevBuf unit_start, unit_size, unit_blk, unit_bounds;
    uint32_t n_units = 0, n_packed = 0;
};

struct Relation {
    uint32_t id = 0, n_rows = 0, n_cols = 0;
    // asynchronous load: copies and validation queued on the copy stream,
    // finished (event wait, validation read back) on first use
    bool pending = false;
    hipEvent_t ready = nullptr;
    DevBuf load_stats;
    Relation() = default;
    Relation(const Relation&) = delete;
    Relation& operator=(const Relation&) = delete;
    ~Relation() {
        if (ready) (void)hipEventDestroy(ready);
    }
    std::vector<Column> cols;
    std::vector<ColDev> h_cols;
    DevBuf d_cols;
    std::map<std::pair<uint32_t, uint32_t>, GramIndex> grams;
    std::map<uint32_t, DevBuf> char_sig;
    std::map<uint32_t, Partition> parts;
    std::map<std::vector<uint32_t>, uint64_t> composite;
};

struct RuleSet {
    uint32_t id = 0, rel_id = 0;
    std::vector<hb_pred> distinct;
    std::vector<std::vector<uint32_t>> rules;  // distinct predicate ids per rule, input order
    std::vector<uint32_t> keys;                // blocking-key attributes, first-appearance order
    bool ordered = false;                      // a predicate tells t from s: ordered output
    std::vector<double> sp, cost;
    std::vector<std::vector<uint64_t>> buckets;
    std::vector<uint64_t> bucket_n;
    bool partitioned = false;
    uint64_t candidates = 0;
    bool has_result = false;
    int result_plan = -1;
    DevBuf result;
    uint64_t n_result = 0;
};

// The cost-model MLP (16 -> 64 -> 64 -> 2): fp32 master parameters and
// Adam moments on the device.
struct CostModel {
    bool ready = false;
    uint64_t adam_t = 0;
    DevBuf params, m, v;
};

struct ProfEntry {
    double ms = 0.0;
    uint64_t launches = 0;
    double bytes = 0.0;   // algorithmic HBM bytes of the launches
};

struct Pending {
    std::string name;
    hipEvent_t a, b;
    double bytes = 0.0;
};

struct Batch;   // batched matching (hb_batch.cpp)

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t copy_stream = nullptr;   // asynchronous loads (created on first use)
    hb_alloc_fn alloc_fn = nullptr;
    hb_free_fn free_fn = nullptr;
    void* user = nullptr;
    std::string err;
    uint32_t next_id = 1;
    std::map<uint32_t, std::unique_ptr<Relation>> rels;
    std::map<uint32_t, std::unique_ptr<RuleSet>> rulesets;
    bool profiling = false;
    std::map<std::string, ProfEntry> prof;
    std::vector<Pending> pending;
    hb_match_stats last{};
    uint32_t lds_limit = 0;
    uint32_t rows_per_wave = 64;   // i-rows per wave batch of hb_match's launches (16, 32 or 64)
    uint32_t sparse_rows = 0;      // the per-lane form's threshold (0: the default of the batch size)
    float learned_min_saving = 0.25f;   // predicted saving a key partition's per-block plans must reach
    bool pack_small_blocks = false;     // hb_set_pack_small_blocks
    CostModel model;        // per (block, predicate): the learned plan's model
    CostModel pair_model;   // per (predicate, pair): the estimated cost's network
    int model_sel = 0;      // HB_MODEL_BLOCK / HB_MODEL_PAIR: what hb_costmodel_* act on
    // hb_set_cost_estimate: the rule set's predicate costs from the static
    // per-operator formulas (0) or from the pair network over sampled pairs
    int cost_source = 0;
    uint32_t cost_samples = 1024;
    uint64_t cost_seed = 0x48425041ull;
    std::map<uint32_t, std::shared_ptr<Batch>> batches;
    // the last autotuned batch launch form, reused by batches created
    // without autotuning
    bool batch_tuned = false;
    int tuned_form = 0;
    uint32_t tuned_grab = 0, tuned_occupancy = 1;
    // the device's scratch array of the allocation-free entry point (its
    // address on this device, or null with the reason in scratch_err)
    uint8_t* scratch = nullptr;
    std::string scratch_err;
    // arena mode: while `arena` is set, every DevBuf::alloc takes the next
    // 256-byte-aligned piece of [arena, arena + arena_cap) and no buffer is
    // freed; the owner of the arena resets it when its call ends
    uint8_t* arena = nullptr;
    size_t arena_cap = 0, arena_used = 0;

    void* arena_take(size_t bytes) {
        const size_t at = (arena_used + 255) & ~(size_t)255;
        if (bytes > arena_cap || at > arena_cap - bytes)
            fail(HB_ERR_LIMIT, "the call needs more than the " + std::to_string(arena_cap) +
                                   " bytes of the scratch array (" + std::to_string(at + bytes) + " asked)");
        arena_used = at + bytes;
        return arena + at;
    }

    void* raw_alloc(size_t bytes) {
        if (bytes == 0) bytes = 16;
        void* p = nullptr;
        if (alloc_fn) {
            p = alloc_fn(bytes, user);
        } else {
            if (hipMallocAsync(&p, bytes, stream) != hipSuccess) p = nullptr;
        }
        if (!p) fail(HB_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
        if (reinterpret_cast<uintptr_t>(p) & 15) {   // kernels read 16-byte words and aligned dwords
            raw_free(p);
            fail(HB_ERR_OOM, "the allocator returned a block not aligned to 16 bytes");
        }
        return p;
    }
    void raw_free(void* p) {
        if (!p) return;
        if (free_fn) free_fn(p, user);
        else (void)hipFreeAsync(p, stream);
    }

    // `bytes`: the launch's algorithmic HBM bytes (each input it must read
    // once, each output it must write once)
    template <typename F>
    void timed(const char* name, F&& launch, double bytes = 0.0) {
        if (!profiling || arena) {   // no events inside an allocation-free call
            HB_HIP(launch());
            return;
        }
        Pending pd;
        pd.name = name;
        pd.bytes = bytes;
        HB_HIP(hipEventCreate(&pd.a));
        HB_HIP(hipEventCreate(&pd.b));
        HB_HIP(hipEventRecord(pd.a, stream));
        HB_HIP(launch());
        HB_HIP(hipEventRecord(pd.b, stream));
        pending.push_back(pd);
    }
    // Host wall time of a step (including any synchronisation it does).
    template <typename F>
    void host_timed(const char* name, F&& work) {
        if (!profiling) {
            work();
            return;
        }
        const auto t0 = std::chrono::steady_clock::now();
        work();
        auto& e = prof[name];
        e.ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        e.launches += 1;
    }
    void drain_profile() {
        for (auto& pd : pending) {
            (void)hipEventSynchronize(pd.b);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, pd.a, pd.b);
            auto& e = prof[pd.name];
            e.ms += ms;
            e.launches += 1;
            e.bytes += pd.bytes;
            (void)hipEventDestroy(pd.a);
            (void)hipEventDestroy(pd.b);
        }
        pending.clear();
    }
    void sync() { HB_HIP(hipStreamSynchronize(stream)); }
};

inline void DevBuf::alloc(Ctx* c, size_t bytes) {
    release();
    c_ = c;
    if (c->arena) {
        p_ = c->arena_take(bytes == 0 ? 16 : bytes);
        borrowed_ = true;
    } else {
        p_ = c->raw_alloc(bytes);
    }
    n_ = bytes;
}

inline void DevBuf::release() {
    if (p_ && c_ && !borrowed_) c_->raw_free(p_);
    p_ = nullptr;
    n_ = 0;
    c_ = nullptr;
    borrowed_ = false;
}

template <typename T>
inline T read1(Ctx* c, const T* dptr) {
    T v{};
    HB_HIP(hipMemcpyAsync(&v, dptr, sizeof(T), hipMemcpyDeviceToHost, c->stream));
    c->sync();
    return v;
}

// Clears device memory with the library's own fill kernel (usable under
// stream capture, unlike a runtime memset node).
inline void zero(Ctx* c, void* p, size_t bytes) { HB_HIP(launch_zero_bytes(p, bytes, c->stream)); }

void finish_load(Ctx* c, Relation& rel);   // hb_api.cpp

inline Relation& get_rel(Ctx* c, uint32_t id) {
    auto it = c->rels.find(id);
    if (it == c->rels.end()) fail(HB_ERR_STALE_ID, "unknown relation id " + std::to_string(id));
    if (it->second->pending) finish_load(c, *it->second);
    return *it->second;
}

inline RuleSet& get_rs(Ctx* c, uint32_t id, uint32_t rel_id) {
    auto it = c->rulesets.find(id);
    if (it == c->rulesets.end()) fail(HB_ERR_STALE_ID, "unknown rule set id " + std::to_string(id));
    if (it->second->rel_id != rel_id) fail(HB_ERR_STALE_ID, "rule set was compiled for another relation");
    return *it->second;
}

inline int bit_width(uint64_t v) {
    int b = 0;
    while (v) { ++b; v >>= 1; }
    return b;
}

inline std::vector<int> shifts_for_bits(int bits, int base) {
    std::vector<int> s;
    for (int x = 0; x < bits; x += 8) s.push_back(base + x);
    return s;
}

// Address of this device's copy of the allocation-free entry point's
// scratch array (hb_noalloc.hip); the device must be current.  Null, with
// the reason in *err, when the runtime cannot give it.
uint8_t* scratch_address(int device, std::string* err);

// cost models (hb_learn.cpp): the hb_costmodel_* calls act on the
// selected model; model_forward runs a given one on device rows
CostModel& selected_model(Ctx* c);
void model_forward(Ctx* c, const CostModel& m, const float* x, uint64_t n, float* y);
void costmodel_init(Ctx* c, uint64_t seed);
void costmodel_set(Ctx* c, const float* p, uint32_t n);
void costmodel_get(Ctx* c, float* p, uint32_t n);
void costmodel_train(Ctx* c, const float* x, const float* t, uint64_t n, int on_device, uint32_t epochs,
                     uint32_t batch, float lr, float* final_loss);
void costmodel_predict(Ctx* c, const float* x, uint64_t n, int on_device, float* y, int y_on_device);
void costmodel_trace(Ctx* c, const float* x, const float* t, uint32_t n, float* out, uint64_t out_len);
void costmodel_adam(Ctx* c, const float* grad_host, float lr);
void costmodel_save(Ctx* c, const char* path);
void costmodel_load(Ctx* c, const char* path);

}  // namespace hb
