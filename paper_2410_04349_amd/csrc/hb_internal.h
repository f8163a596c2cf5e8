// Internal declarations of libhb: device descriptors, plan bytecode, launch
// wrappers.  Shared by the host code and the HIP kernels of this library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace hb {

constexpr int kTile = 64;        // tuples per tile side (one wave of j's)
constexpr int kRows = 16;        // i-rows per wave batch (four batches per 64-row tile)
// A filter step runs per lane, live row by live row, when no lane has more
// live rows than the threshold (capped at half the batch's rows): the
// context's setting (hb_set_sparse_rows), or 0 for the default of the batch
// size.
constexpr int kMaxSparseRows = 32;
constexpr uint32_t kPackRows = 32;   // blocks of at most this many rows are packed into shared windows
constexpr uint32_t kPackedUnit = 1u << 31;   // unit_size flag of a packed window
__host__ __device__ constexpr uint32_t sparse_rows(uint32_t setting, uint32_t rows) {
    return setting ? setting : rows >= 64 ? 16u : rows >= 32 ? 8u : 4u;
}
constexpr uint64_t kMaxTiles = (1ull << 30) - 8;   // one launch's grid: 4 x tiles, rounded up to 32 < 2^32
constexpr int kLshK = 1024;      // LSH buckets of the selectivity estimate
constexpr int kMaxIntRes = 16;   // int attributes staged per tile
constexpr int kMaxStrRes = 8;    // string attributes staged per tile
constexpr int kMaxGramRes = 8;   // (attribute, q) gram lists staged per tile
constexpr int kMaxPrevKeys = 3;
constexpr int kMaxEdWords = 4;   // 256-byte edit-distance patterns
constexpr uint32_t kLongSigWords = 4;   // q-gram signature words of attributes past 64 windows
constexpr int kMaxPlan = 1536;   // steps of one key's plan
constexpr int kCountPairs = 8 * 4;             // instrumented counters: 8 op kinds x 4, then pairs
constexpr int kCountSlots = kCountPairs + 1;

enum ColType : int32_t { COL_STRING = 0, COL_CATEGORICAL = 1, COL_INT64 = 2 };

// One column in device memory.
struct ColDev {
    int32_t type;
    uint32_t max_len;        // STRING: longest value in bytes
    const uint64_t* off;     // STRING: n+1 offsets
    const uint8_t* bytes;    // STRING
    const int64_t* values;   // CATEGORICAL / INT64
    const uint8_t* valid;    // LSB-first bitmap or nullptr
};

// Sorted distinct q-gram codes of one (string attribute, q).
// Row r's list starts at off[r] and holds cnt[r] codes, ascending.  A
// non-empty string shorter than q has cnt = 1, flag bit 0 set, and the code
// (len << 24) | big-endian bytes; the empty string has cnt = 0.
struct GramDev {
    const uint64_t* off;
    const uint32_t* cnt;
    const uint32_t* codes;
    const uint8_t* flags;
    uint32_t q;
    uint32_t max_cnt;   // bound on a row's code count: the longest row's window count
    uint32_t attr;
    uint32_t sig_words;   // 64-bit words of a row's q-gram signature (1, or 4 past 64 windows)
    uint32_t sig_col;     // first f64 feature column of the signature, counted from the first gram column
    uint32_t pad;
};

// Plan operations.  Filters are exact necessary conditions of the
// predicate they precede (a filter that fails proves the predicate false);
// the verify operations compute the predicate itself.
enum Op : uint8_t {
    OP_EQ_INT = 0,   // value equality (categorical / int64)
    OP_ABSDIFF = 1,  // |a - b| <= d
    OP_EQF = 2,      // string equality filter: equal length and character signature
    OP_EDF = 3,      // edit distance filter: |m - n| <= k and signature bound <= k
    OP_JACF = 4,     // Jaccard filter: q-gram signature bound on the intersection
    OP_EQ_STR = 5,   // verify: byte equality
    OP_ED = 6,       // verify: Levenshtein distance <= k (Myers)
    OP_JAC = 7,      // verify: q-gram Jaccard >= num / den (merge intersection)
    OP_CP = 8,       // rule end: the pair has a witness
    // predicates that tell t from s (ordered rule sets only; the pair's two
    // valuations get a mask each)
    OP_CONST = 9,    // t.A = c (aux 0) or s.A = c (aux 1); param = c
    OP_XEQ = 10,     // t.A = s.B: res = A, aux = B (both int resources)
    OP_XED = 11,     // Levenshtein(t.A, s.B) <= k: res = A, aux = B (string resources), param = k
    // a first-stage step shared by consecutive rules (the execution tree's
    // shared edge, Section 4.2): OP_GUARD evaluates the step whose operation
    // is in `aux` once, and the rules up to the OP_ENDGUARD at `cp` start
    // from the pairs that pass it; OP_ENDGUARD returns to every pair
    OP_GUARD = 12,
    OP_ENDGUARD = 13,
    // q-gram Jaccard(t.A, s.B) >= num / den (ordered rule sets): res = A,
    // aux = B (gram resources of one q), param = (num << 32) | den
    OP_XJAC = 14,
    // q-gram containment of t.A in s.B >= num / den (asymmetric; ordered
    // rule sets; A may be B): operands as OP_XJAC
    OP_XCONT = 15
};

// One step of the sequential execution path.  `slot` identifies the step
// (distinct predicates 0..63, their filters 64..127); `res` indexes the
// int / string / gram resource it reads; `cp` is the index of the
// checkpoint that closes the rule.
// `param` is d (|a - b| <= d), k (edit distance) or (num << 32) | den
// (Jaccard threshold num / den).
struct Instr {
    uint8_t op;
    uint8_t slot;
    uint8_t res;
    uint8_t aux;    // OP_CONST: side; OP_XEQ, OP_XED, OP_XJAC, OP_XCONT: resource of B
    uint16_t cp;
    uint16_t pad1;
    uint64_t param;
};
static_assert(sizeof(Instr) == 16, "Instr layout");

// Block-major feature columns of one key partition (structure of arrays,
// position p = p-th row of the key-sorted permutation):
//   f64[(x) * n + p]: x < n_int: int value; then n_str character signatures;
//                     then the q-gram signatures, sig_words columns per gram
//                     resource (word w of resource r at column
//                     n_int + n_str + gram[r].sig_col + w)
//   f32[(x) * n + p]: x = 0: row id; 1: validity mask (bit r: int resource r,
//                     16 + r: string resource r, 24 + r: gram resource r);
//                     then n_str lengths; then n_gram set sizes (bit 31:
//                     short-string flag); then n_gram Jaccard-filter words
//                     ((|A| - popcount(signature words)) << 16 | |A|, and 1 for a
//                     missing value, whose signature is 0: with a threshold
//                     above 0 that word fails the filter against anything)
struct Features {
    const uint64_t* f64;
    const uint32_t* f32;
    uint64_t n;       // column stride: positions (rows with a valid key) + kTile zeroed
                      // pad positions, so a 16-row batch and a 64-lane j-tile read
                      // in bounds
};

// Everything the match kernel needs for one (relation, key partition, plan).
struct MatchParams {
    const ColDev* cols;
    Features feat;
    // partition of the key: blocks of >= 2 rows
    const uint32_t* blk_start;
    const uint32_t* blk_size;
    // the match's work units: blocks, or windows of consecutive small
    // blocks packed into one tile.  With unit_start null the units are the
    // blocks; otherwise unit u spans unit_size[u] positions from
    // unit_start[u] (bit 31 of the size: a packed window), unit_blk[u] is
    // its block (~0u for a window) and bit k of unit_bounds[u] marks
    // position k of a window as the last of its block (or a lone row)
    const uint32_t* unit_start;
    const uint32_t* unit_size;
    const uint32_t* unit_blk;
    const uint64_t* unit_bounds;
    const uint64_t* tile_prefix;   // units + 1 entries
    const uint32_t* tile_blk;      // unit of each tile (n_tiles entries)
    uint32_t n_blocks;
    uint32_t ordered;   // 1: the rule set tells t from s (both valuations of a pair, ordered output)
    uint64_t n_tiles;
    // plan
    const Instr* plan;
    uint32_t plan_len;
    uint32_t n_int, n_str, n_gram, n_prev;
    uint32_t int_attr[kMaxIntRes];
    uint32_t str_attr[kMaxStrRes];
    GramDev gram[kMaxGramRes];
    uint32_t prev_res[kMaxPrevKeys];   // int resources of earlier keys (canonical owner)
    uint32_t ed_words;                 // 64-bit words of the pattern-match table (0: no edit distance)
    // LDS layout (byte offsets into dynamic shared memory)
    uint32_t lds_wave_stride;          // bytes of the wave's region (from offset 0)
    uint32_t lds_wave_peq, lds_wave_myers, lds_wave_igram[kMaxGramRes];
    uint32_t lds_bytes;
    // output
    uint64_t* out;
    uint64_t cap;
    unsigned long long* counter;
    // instrumented pass only: per operation kind {wave-steps, lanes, lanes
    // passed, work units}, then pairs evaluated; nullptr in the normal pass
    unsigned long long* counts;
    uint32_t lds_counts;
    // per-block plans (learned): block b runs the plan_len instructions at
    // plan + blk_slot[b] * plan_len; blk_slot == nullptr: one plan for every
    // block
    const uint32_t* blk_slot;
    // i-rows per wave batch of the plain launch: 16 (four batches per tile),
    // 32 (two) or 64 (one); ordered rule sets and the batch kernels use 16
    uint32_t rows;
    // the per-lane form's threshold setting (0: the default of the batch size)
    uint32_t sparse_rows;
    // 1: no attribute the plan reads has a missing value (the validity mask
    // words are not read)
    uint32_t all_valid;
};

// Gather of the block-major feature columns: grid.y = 1 + n_int + n_str +
// n_gram slices (row id and validity mask, then one per resource), each
// thread one (position, slice), with every column's pointers given
// directly so a thread's loads depend only on its row.
struct GatherParams {
    const uint32_t* perm;
    uint64_t n;           // positions
    uint64_t stride;      // column stride (>= n; positions n .. stride - 1 are zeroed)
    uint32_t n_int, n_str, n_gram;
    const uint8_t* int_valid[kMaxIntRes];     // nullptr: every row valid
    const int64_t* int_vals[kMaxIntRes];
    const uint8_t* str_valid[kMaxStrRes];
    const uint64_t* str_off[kMaxStrRes];
    const uint64_t* csig[kMaxStrRes];
    const uint8_t* gram_valid[kMaxGramRes];
    const uint32_t* gram_cnt[kMaxGramRes];
    const uint8_t* gram_flags[kMaxGramRes];
    const uint64_t* gsig[kMaxGramRes];        // sig_words words per row
    uint32_t gram_words[kMaxGramRes], gram_col[kMaxGramRes];
    uint64_t* f64;
    uint32_t* f32;
    // row records (the two-pass gather): n_rows records of rec_words u32
    // words each, in row order: the row's f64 features (two words each,
    // in column order), then its f32 features from column 1 on (validity
    // mask, lengths, q-gram counts, filter words), zero-padded to a
    // multiple of four words
    uint32_t* rec;
    uint32_t n_rows, rec_words, n64, n32;
};

// ---------------------------------------------------------------- launches
// Each returns hipSuccess or the launch error.  All run on `s`.

// max length / total bytes / monotonic check of string offsets
hipError_t launch_string_stats(const uint64_t* off, uint32_t n, uint32_t* d_max_len,
                               unsigned long long* d_total, uint32_t* d_bad, hipStream_t s);
// min / max of int64 values over valid rows (as order-preserving u64)
hipError_t launch_minmax_u64(const int64_t* vals, const uint8_t* valid, uint32_t n,
                             unsigned long long* d_min, unsigned long long* d_max,
                             unsigned int* d_nvalid, hipStream_t s);

// exclusive scan of n values; tmp must hold scan_tmp_elems(n) elements
size_t scan_tmp_elems(size_t n);
hipError_t launch_exclusive_scan_u32(const uint32_t* in, uint32_t* out, size_t n, uint32_t* tmp,
                                     hipStream_t s);
hipError_t launch_exclusive_scan_u64(const uint64_t* in, uint64_t* out, size_t n, uint64_t* tmp,
                                     hipStream_t s);

// LSD radix sort of (u64 key, u32 value) by 8-bit digits at the given shifts.
// Sorts keys/vals in place using the alternate buffers; returns in
// *result_in_alt whether the result ended in the alternate buffers.
size_t radix_tmp_bytes(uint32_t n);
hipError_t radix_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt,
                            uint32_t n, const int* shifts, int n_shifts, void* tmp,
                            bool* result_in_alt, hipStream_t s);

// partition helpers
hipError_t launch_key_extract(const int64_t* vals, const uint8_t* valid, uint32_t n,
                              unsigned long long key_min, uint64_t* keys, uint32_t* rows,
                              const uint32_t* dest, hipStream_t s);
hipError_t launch_valid_flags(const uint8_t* valid, uint32_t n, uint32_t* flags, hipStream_t s);
hipError_t launch_multi_valid_flags(const ColDev* cols, const uint32_t* attrs, uint32_t n_attrs,
                                    uint32_t n, uint32_t* flags, hipStream_t s);
hipError_t launch_gather_key(const ColDev* cols, uint32_t attr, unsigned long long key_min,
                             const uint32_t* rows, uint32_t n, uint64_t* keys, hipStream_t s);
hipError_t launch_compact_rows(const uint32_t* flags, const uint32_t* dest, uint32_t n,
                               uint32_t* rows, hipStream_t s);
// flags[b] = size[b] >= min
// tile_blk[t] = block holding tile t (the last b with tile_prefix[b] <= t)
hipError_t launch_tile_blocks(const uint64_t* tile_prefix, uint32_t n_blocks, uint64_t n_tiles, uint32_t* tile_blk,
                              hipStream_t s);
hipError_t launch_size_flags(const uint32_t* size, uint32_t n, uint32_t min, uint32_t* flags, hipStream_t s);
hipError_t launch_group_heads(const ColDev* cols, const uint32_t* attrs, uint32_t n_attrs,
                              const uint32_t* rows, uint32_t n, uint32_t* head, hipStream_t s);
hipError_t launch_group_sizes(const uint32_t* head, const uint32_t* gid, uint32_t n,
                              uint32_t n_groups, uint32_t* start, hipStream_t s);
hipError_t launch_block_table(const uint32_t* gstart, uint32_t n_groups, uint32_t n_rows,
                              const uint32_t* dest, uint32_t* blk_start, uint32_t* blk_size,
                              uint64_t* tiles, unsigned long long* pairs, hipStream_t s);
hipError_t launch_group_pairs(const uint32_t* gstart, uint32_t n_groups, uint32_t n_rows,
                              unsigned long long* pairs, hipStream_t s);
hipError_t launch_ge2_flags(const uint32_t* gstart, uint32_t n_groups, uint32_t n_rows,
                            uint32_t* flags, hipStream_t s);

// q-gram index
hipError_t launch_gram_slots(const ColDev* col, uint32_t n, uint32_t q, uint64_t* slots,
                             hipStream_t s);
// max_windows: the largest L - q + 1 of the column (<= 4096; picks the
// sort: registers up to 64 windows, a wave's LDS beyond).  Also writes each
// row's q-gram signature (bit mix64(code) mod 64 W set for every distinct
// code): W = 1 word per row up to 64 windows, kLongSigWords beyond.
hipError_t launch_gram_build(const ColDev* col, uint32_t n, uint32_t q, const uint64_t* off,
                             uint32_t* codes, uint32_t* cnt, uint8_t* flags, uint64_t* sig, uint32_t max_windows,
                             hipStream_t s);

// character-presence signature of every string of a column
hipError_t launch_char_sig(const ColDev* col, uint32_t n, uint64_t* sig, hipStream_t s);
// block-major feature columns, read column by column at the permuted rows
// (no temporary; for allocation-free calls)
hipError_t launch_gather_features(const GatherParams& p, hipStream_t s);
// the same columns in two passes: each row's features packed into its
// record in row order (sequential reads), then whole records moved to the
// permuted positions and split into columns (p.rec holds the records)
hipError_t launch_pack_records(const GatherParams& p, hipStream_t s);
hipError_t launch_gather_records(const GatherParams& p, hipStream_t s);

// LSH bucket histogram of one predicate (op, q, d) over column `col`
hipError_t launch_lsh_hist(const ColDev* col, uint32_t n, int op, uint32_t q, int64_t d,
                           unsigned long long* hist, hipStream_t s);

// the match kernel
hipError_t launch_match(const MatchParams& p, hipStream_t s);

// ------------------------------------------------------------ learned plan
// One distinct predicate of a key plan, as evaluated in isolation by the
// logging pass and described by the block-feature pass.  `op` is the plan
// operation that decides it (OP_EQ_INT, OP_ABSDIFF, OP_EQ_STR, OP_ED,
// OP_JAC); `res` its resource; `param` as in Instr.
struct PredSpec {
    uint8_t op;
    uint8_t res;
    uint16_t pred;     // distinct predicate id in the rule set
    uint8_t aux;       // as Instr::aux
    uint8_t pad[3];
    uint64_t param;
};
constexpr int kMaxSpecs = 64;
constexpr uint32_t kFeatureSample = 256;   // positions per block the features are computed on
constexpr int kFeatures = 16;

struct LearnParams {
    MatchParams mp;                  // columns, features, blocks, resources, LDS layout
    PredSpec spec[kMaxSpecs];
    uint32_t n_spec;
    uint32_t samples;                // logging: sampled waves per block
    uint64_t seed;
    float* features;                 // [n_list x n_spec x 16]
    const uint32_t* blocks;          // features of blocks[0 .. n_list); nullptr: every block
    uint32_t n_list;
    unsigned long long* counts;      // logging: [n_blocks x n_spec x 4] {lanes, passed, cycles, first step passed}
};
hipError_t launch_block_features(const LearnParams& p, hipStream_t s);
hipError_t launch_log_samples(const LearnParams& p, hipStream_t s);

// ------------------------------------------------------------ per-pair cost network
// The estimated cost of Section 4.2 ("Evaluation cost", "Estimated cost"):
// sampled pairs of D x D (not of blocks), each described to the per-pair
// network by 16 features of the predicate and the two A-values, read
// straight from the relation's columns.  Pair s of a seed:
// i = mix64(seed + 2s) mod n, j = mix64(seed + 2s + 1) mod n, j = (i + 1)
// mod n when equal to i.  Rows are predicate-major: row x * samples + s.
enum PairKind : uint8_t { PK_VALUE_EQ = 0, PK_ABSDIFF = 1, PK_STRING_EQ = 2, PK_EDIT = 3, PK_JACCARD = 4 };
struct PairSpec {
    uint8_t kind;       // PairKind
    uint8_t gram;       // PK_JACCARD: index into PairParams::gram
    uint16_t pad;
    uint32_t attr;      // the compared attribute
    uint32_t q;         // PK_JACCARD
    uint32_t k;         // PK_EDIT: distance bound
    int64_t d;          // PK_ABSDIFF
    uint32_t num, den;  // PK_JACCARD: threshold num / den
};
constexpr uint32_t kPairLdsPeq = 0;                                   // 256 x 4 64-bit words
constexpr uint32_t kPairLdsMyers = 256 * kMaxEdWords * 8;             // long-pattern state
constexpr uint32_t kPairLdsGrams = kPairLdsMyers + 2 * kMaxEdWords * 64 * 8;   // row i's q-gram list
struct PairParams {
    const ColDev* cols;             // the relation's columns (device)
    GramDev gram[kMaxGramRes];
    PairSpec spec[kMaxSpecs];
    uint32_t n_spec, samples, n_rows;
    uint32_t lds_bytes;             // logging: kPairLdsGrams + the longest q-gram list
    uint64_t seed;
    float* features;                // [n_spec x samples x 16]
    float* y;                       // estimate: the network's outputs [n_spec x samples x 2]
    double* sums;                   // estimate: [n_spec] summed cycles
    uint8_t* sat;                   // logging: [n_spec x samples] the check's result
    unsigned long long* cycles;     // logging: [n_spec x samples] clock cycles of the check
    uint32_t* pairs;                // logging: [samples x 2] (i, j), or nullptr
};
hipError_t launch_pair_log(const PairParams& p, hipStream_t s);
hipError_t launch_pair_features(const PairParams& p, hipStream_t s);
hipError_t launch_pair_sum(const PairParams& p, hipStream_t s);

// Per-block plan choice from the cost model's outputs.  Rules keep the
// heuristic path's order; per block and rule the kernel picks the first-stage
// order and the verification order.  Equal choices share a plan slot of an
// open-addressing table keyed by a hash of the choice; the first block to
// claim a slot writes that slot's plan by permuting the heuristic plan inside
// each rule's segment (segments keep their positions, so checkpoint targets
// are unchanged).  Slot 0 is the heuristic plan, also taken by blocks not in
// the list and when the table is full.
constexpr int kMaxPlanRules = 64;
constexpr int kMaxRuleSteps = 10;
// Distinct plans of a partition (power of two): a wave fetches its plan's
// steps through the scalar cache, and many distinct copies of a long plan
// cost more in fetch misses than their orders save
constexpr uint32_t kPlanSlots = 256;
struct PlanChoiceParams {
    const float* y;                   // [n_blocks x n_spec x 2] model outputs, in list order
    const uint32_t* blocks;           // the listed blocks (the rest keep slot 0)
    const uint32_t* blk_size;
    uint32_t n_blocks, n_spec;        // n_blocks: list length
    uint32_t n_rules;                 // rules of the partition's plan, in heuristic order
    uint32_t n_slots;                 // table size (power of two, <= kPlanSlots)
    uint32_t plan_len;                // instructions of one plan
    uint32_t rows;                    // i-rows per wave batch of the launch (16, 32 or 64)
    uint32_t sparse_rows;             // the per-lane form's threshold setting (0: default)
    uint8_t rule_len[kMaxPlanRules];  // first-stage steps per rule (a shared guard step excluded)
    uint16_t rule_seg[kMaxPlanRules]; // first instruction of each rule's segment
    uint8_t rule_guard[kMaxPlanRules];   // spec index of the rule's shared guard step, 0xFF: none
    uint8_t rule_spec[kMaxPlanRules][kMaxRuleSteps];   // spec index of each step, heuristic order
    uint8_t spec_kind[kMaxSpecs];     // plan operation of each spec (Op)
    unsigned long long* keys;         // [n_slots] choice hash per slot, 0 = empty
    Instr* code;                      // [n_slots x plan_len]; slot 0 holds the heuristic plan
    uint32_t* blk_slot;               // [n_blocks] out
    unsigned long long* stats;        // [3] blocks with a learned plan, blocks over capacity, plans written
    float* cost;                      // [2] predicted cost of the listed blocks: heuristic plan, chosen plans
};
hipError_t launch_plan_choice(const PlanChoiceParams& p, hipStream_t s);

// Persistent work-stealing matching over n_parts partitions (device array
// mps, tile prefix over them, total items); `cursor` must be zero at launch.
hipError_t launch_match_persistent(const MatchParams* mps, const uint64_t* prefix, uint32_t n_parts, uint64_t total,
                                   unsigned long long* cursor, uint32_t grab, uint32_t grid, uint32_t lds_bytes,
                                   hipStream_t s);
hipError_t match_persistent_occupancy(uint32_t lds_bytes, int* blocks_per_cu);
// One workgroup per work item over the same queue (total < 2^31).
hipError_t launch_match_multi(const MatchParams* mps, const uint64_t* prefix, uint32_t n_parts, uint64_t total,
                              uint32_t lds_bytes, hipStream_t s);
// p[0 .. n) = v (a kernel, so it may be captured in a graph)
hipError_t launch_fill_u64(unsigned long long* p, uint64_t n, unsigned long long v, hipStream_t s);
// bytes [p, p + n) = 0 (a kernel)
hipError_t launch_zero_bytes(void* p, size_t n, hipStream_t s);

// ------------------------------------------------------------ cost model
// C[M x N] = op(A) op(B) (+ bias[N]); op(X) = X or X^T (row-major storage
// with leading dimension ld); where `mask` is given, entries with
// mask[i][j] <= 0 become 0; where `relu` is given it receives max(C, 0).
struct GemmArgs {
    const float* A;
    const float* B;
    float* C;
    const float* bias;
    const float* mask;
    float* relu;
    int M, N, K;
    int lda, ldb, ldc;
    int transA, transB;
};
hipError_t launch_gemm(const GemmArgs& g, hipStream_t s);
// y [n x 2] = the cost model on x [n x 16] (inference only, one kernel)
hipError_t launch_mlp_forward(const float* W, const float* x, uint64_t n, float* y, hipStream_t s);
hipError_t launch_colsum(const float* A, int rows, int cols, float* out, hipStream_t s);
hipError_t launch_mse_grad(const float* Y, const float* T, int n, float scale, float* dY, float* sse,
                           hipStream_t s);
hipError_t launch_adam(float* w, const float* g, float* m, float* v, int n, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s);

// write pairs in order: out[x] = in[x] (device copy helper for the result)
hipError_t launch_copy_u64(const uint64_t* in, uint64_t* out, uint64_t n, hipStream_t s);

}  // namespace hb
