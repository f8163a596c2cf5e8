/*
 * hb.h -- C ABI of the MI355X rule-based blocking library (libhb.so).
 *
 * The library computes, for a relation D and a set Delta of matching
 * dependencies (MDs), the set Ca(D) of tuple pairs (t_i, t_j) for which some
 * MD in Delta is a witness: every predicate of its precondition holds
 * (Section 2, "Rule-based blocking"; the problem statement of Section 2,
 * "Our scope: blocking": relation plus rules in, candidate pairs out).
 *
 * Conventions shared by every call:
 *   - Every call returns an hb_status; nothing throws across the ABI.
 *     On failure hb_last_error(ctx) describes the cause and the context
 *     stays usable.
 *   - Inputs are copied (or, for device inputs, read) during the call; the
 *     caller may free or reuse them when the call returns.
 *   - Device memory comes from the allocator given to hb_create (or
 *     hipMallocAsync on the context stream when none is given) and is
 *     released by hb_release_relation / hb_destroy.
 *   - All device work runs on the stream given to hb_create (or a stream the
 *     context creates).  Calls that return host-visible results synchronise
 *     that stream before returning.
 *   - A context is not thread-safe: serialise calls on one context.
 *   - Rows are 0-based positions in the arrays given to hb_load_relation.
 */
#ifndef HB_H
#define HB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hb_ctx hb_ctx;

typedef enum {
    HB_OK = 0,
    HB_ERR_INVALID_ARG = 1,  /* NULL pointer, bad size, bad enum, bad offsets */
    HB_ERR_TYPE = 2,         /* predicate applied to an attribute of the wrong type */
    HB_ERR_UNBLOCKABLE = 3,  /* a rule has no equality on a categorical/int64 attribute */
    HB_ERR_LIMIT = 4,        /* a documented size limit is exceeded */
    HB_ERR_OOM = 5,          /* the allocator returned NULL */
    HB_ERR_CAPACITY = 6,     /* output buffer too small; *n_pairs holds the size needed */
    HB_ERR_HIP = 7,          /* a HIP runtime call failed */
    HB_ERR_STALE_ID = 8,     /* relation / rule-set id unknown or released */
    HB_ERR_STATE = 9         /* call out of order (e.g. hb_match before hb_partition) */
} hb_status;

/* Limits (HB_ERR_LIMIT beyond them). */
#define HB_MAX_RULES 64          /* rules per rule set */
#define HB_MAX_RULE_PREDS 10     /* predicates per rule (the paper's default bound) */
#define HB_MAX_DISTINCT_PREDS 64 /* distinct predicates per rule set */
#define HB_MAX_KEYS 4            /* distinct blocking-key attributes per rule set */
#define HB_MAX_ED_LEN 256        /* longest string of an attribute used by an edit-distance predicate */
#define HB_MAX_GRAM_LEN 4096     /* longest string of an attribute used by a Jaccard predicate */
#define HB_MAX_ED_K 255
#define HB_MAX_Q 4
#define HB_MAX_JACCARD_DEN (1u << 18) /* threshold denominator in lowest terms */

/* Device allocator: return `bytes` bytes of device memory on the context's
 * device, aligned to at least 16 bytes (NULL on failure; a misaligned block
 * fails the call with HB_ERR_OOM); `user` is passed through. */
typedef void* (*hb_alloc_fn)(size_t bytes, void* user);
typedef void (*hb_free_fn)(void* ptr, void* user);

/* Create a context on HIP device `device`.  `alloc`/`free_fn` may both be
 * NULL (then hipMallocAsync/hipFreeAsync on the stream are used).  `stream`
 * is a hipStream_t (NULL: the context creates a non-blocking stream of
 * default priority).  The caller keeps ownership of a given stream. */
hb_status hb_create(hb_ctx** out, int device, hb_alloc_fn alloc, hb_free_fn free_fn,
                    void* user, void* stream);
void hb_destroy(hb_ctx* ctx);
const char* hb_last_error(const hb_ctx* ctx);
const char* hb_version(void);

/* ------------------------------------------------------------ relations
 * A relation D of schema R = (A_1..A_n) (Section 2, "Relations"), stored
 * column-wise.  Table 1's missing values ("-") are expressed with the
 * validity bitmap: a missing value fails every predicate (Example 3; the
 * Section 4 remark on (t1, t5)).
 */
typedef enum { HB_COL_STRING = 0, HB_COL_CATEGORICAL = 1, HB_COL_INT64 = 2 } hb_coltype;

typedef struct {
    int32_t type;            /* hb_coltype */
    const uint64_t* offsets; /* STRING: n_rows + 1 non-decreasing byte offsets, offsets[0] = 0 */
    const uint8_t* bytes;    /* STRING: offsets[n_rows] bytes (may be NULL when that is 0) */
    const int64_t* values;   /* CATEGORICAL (dictionary codes) / INT64: n_rows values */
    const uint8_t* valid;    /* optional LSB-first validity bitmap, ceil(n_rows / 8) bytes;
                                NULL = every value present */
} hb_column;

/* Load a relation.  `on_device` = 0: the column arrays are host memory and
 * are copied to the device; 1: they are device memory of this context's
 * device and are copied device-to-device.  1 <= n_rows < 2^31,
 * 1 <= n_cols <= 256.  String offsets are validated (HB_ERR_INVALID_ARG). */
hb_status hb_load_relation(hb_ctx* ctx, uint32_t n_rows, uint32_t n_cols, const hb_column* cols,
                           int on_device, uint32_t* rel_id);

/* As hb_load_relation, but returns once the copies are queued: they, and
 * the offset validation, run on a second stream of the context, so a
 * relation's host-to-device copy overlaps the matching of relations loaded
 * before it (Section 5's pipeline overlaps transfer and compute).  The
 * relation is finished on its first use by any other call (which waits for
 * its copies); invalid offsets are reported there (HB_ERR_INVALID_ARG, the
 * relation stays releasable).  The caller's arrays must stay valid and
 * unchanged until then; host arrays should be pinned (hipHostMalloc) for
 * the copy to be asynchronous. */
hb_status hb_load_relation_async(hb_ctx* ctx, uint32_t n_rows, uint32_t n_cols, const hb_column* cols,
                                 int on_device, uint32_t* rel_id);
/* Release a relation and every rule set compiled against it. */
hb_status hb_release_relation(hb_ctx* ctx, uint32_t rel_id);

/* ------------------------------------------------------------ rules
 * Predicates of the forms t.A = s.A, t.A ~ s.A, t.A = c and t.A = s.B
 * (Section 2, "Predicates"); a valuation binds t to a pair's first tuple and
 * s to its second (Section 2, "Semantics").  The operators:
 *   HB_EQ          byte-exact equality (STRING) or value equality
 *                  (CATEGORICAL, INT64);
 *   HB_ED_LE       Levenshtein distance over bytes <= k        (STRING);
 *   HB_JACCARD_GE  |G_q(a) & G_q(b)| * den >= num * |G_q(a) | G_q(b)|, G_q the
 *                  set of distinct length-q byte windows, {s} for a non-empty
 *                  string shorter than q, empty for the empty string, and
 *                  J(empty, empty) = 1                          (STRING);
 *   HB_ABSDIFF_LE  |a - b| <= d, exact over int64                (INT64);
 *   HB_EQ_CONST    t.A = c (side 0) or s.A = c (side 1): the tuple's value
 *                  is present and equals the int64 constant c
 *                                                   (CATEGORICAL, INT64);
 *   HB_EQ_CROSS    t.A = s.B: t's value of A and s's value of B (attr_b) are
 *                  both present and equal     (CATEGORICAL, INT64 for both);
 *   HB_ED_CROSS_LE t.A ~ s.B: Levenshtein distance over bytes from t's A to
 *                  s's B (attr_b) <= k            (STRING for both);
 *   HB_JACCARD_CROSS_GE  t.A ~ s.B: the HB_JACCARD_GE test between t's
 *                  q-gram set of A and s's of B (attr_b; one q)
 *                                                 (STRING for both);
 *   HB_CONTAIN_GE  t.A ~ s.B, an asymmetric measure (Section 2 allows any
 *                  similarity, symmetric or asymmetric): the share of t's
 *                  q-grams of A found among s's of B (attr_b, which may
 *                  equal attr), |G_q(t.A) & G_q(s.B)| * den >= num *
 *                  |G_q(t.A)|; an empty t set is contained in anything
 *                                                 (STRING for both).
 * A missing value fails every predicate.  A rule set with an HB_EQ_CONST or
 * an HB_CONTAIN_GE, or an HB_EQ_CROSS, HB_ED_CROSS_LE or
 * HB_JACCARD_CROSS_GE over two different attributes, is *ordered*: its two
 * valuations of a pair may differ, and hb_match lists ordered pairs (see
 * there).  HB_EQ_CROSS with attr_b = attr is an equality (unordered), but
 * never a blocking key; HB_ED_CROSS_LE with attr_b = attr is HB_ED_LE, and
 * HB_JACCARD_CROSS_GE with attr_b = attr is HB_JACCARD_GE.
 * A rule (an MD X -> t.eid = s.eid, Section 2, "Rules") is a conjunction;
 * a rule set is their disjunction.  Every rule must contain an HB_EQ on a
 * CATEGORICAL or INT64 attribute: its first one (in the given order) is the
 * rule's blocking key (the partition key of Section 5.3).
 */
typedef enum {
    HB_EQ = 0,
    HB_ED_LE = 1,
    HB_JACCARD_GE = 2,
    HB_ABSDIFF_LE = 3,
    HB_EQ_CONST = 4,
    HB_EQ_CROSS = 5,
    HB_ED_CROSS_LE = 6,
    HB_JACCARD_CROSS_GE = 7,
    HB_CONTAIN_GE = 8
} hb_op;

typedef struct {
    int32_t op;     /* hb_op */
    uint32_t attr;  /* column index */
    int64_t k;      /* HB_ED_LE, HB_ED_CROSS_LE: 0..HB_MAX_ED_K */
    uint32_t q;     /* HB_JACCARD_GE, HB_JACCARD_CROSS_GE, HB_CONTAIN_GE: 1..HB_MAX_Q */
    uint32_t num;   /* the same three: threshold num/den, 0 <= num <= den */
    uint32_t den;   /* the same three: den > 0, <= HB_MAX_JACCARD_DEN in lowest terms */
    int64_t d;      /* HB_ABSDIFF_LE: d >= 0 */
    uint32_t attr_b;  /* HB_EQ_CROSS, HB_ED_CROSS_LE, HB_JACCARD_CROSS_GE, HB_CONTAIN_GE: column index of B */
    int32_t side;     /* HB_EQ_CONST: 0 = t.A = c, 1 = s.A = c */
    int64_t c;        /* HB_EQ_CONST: the constant */
} hb_pred;

typedef struct {
    uint32_t n_preds;
    const hb_pred* preds;
} hb_rule;

/* Validate and compile a rule set against a relation: dedups predicates,
 * builds the q-gram indexes its Jaccard predicates need and the
 * per-predicate selectivity estimates of the heuristic plan (Section 4.2). */
hb_status hb_compile_rules(hb_ctx* ctx, uint32_t rel_id, uint32_t n_rules, const hb_rule* rules,
                           uint32_t* ruleset_id);

/* Partition the relation on the rule set's blocking keys (Section 2,
 * "Data partitioning"; Section 5.3 partitioning by the root edges' keys):
 * groups rows by exact key value.  *n_candidate_pairs receives the exact
 * number of distinct pairs i < j sharing a value of at least one key. */
hb_status hb_partition(hb_ctx* ctx, uint32_t rel_id, uint32_t ruleset_id,
                       uint64_t* n_candidate_pairs);

/* Evaluation order (output-neutral, Section 4):
 *   HB_PLAN_GIVEN      rules and predicates in the given order;
 *   HB_PLAN_HEURISTIC  the execution plan of Section 4.2 (cost-effectiveness
 *                      order, execution tree, edge scores, DFS order); rules
 *                      whose first steps are the same cheap step on the
 *                      same attribute (any threshold) are placed together
 *                      and share one guard step at the loosest threshold;
 *   HB_PLAN_LEARNED    a plan per block from the context's cost model (a
 *                      different plan on each partition, the paper's future
 *                      topic in Section 8), rules as in the heuristic plan:
 *                      per rule, the first-stage steps (value predicates and
 *                      exact filters) ordered to minimise their expected
 *                      cost on the block's wave batch of min(n, rows) x
 *                      min(n, 64) pairs under the model's predicted pass
 *                      rates, each step tried as the first, kept only where
 *                      the model expects it 10% cheaper than the heuristic
 *                      order; the exact checks stay in the heuristic order.
 *                      Blocks of fewer than 64 tuples keep the heuristic
 *                      plan, and so does every block of a key partition
 *                      where the model expects the per-block plans to save
 *                      under 25% in all (hb_set_learned_min_saving).  Built
 *                      on the device; one 8-byte read-back per key
 *                      partition.
 *                      Needs a cost model (HB_ERR_STATE otherwise).
 * The ordering strategies the paper's experiments compare against
 * (Section 6, "Tests on EPG"), for studies; each is output-neutral:
 *   HB_PLAN_CHEAPEST     the execution tree with predicates ranked cheapest
 *                        first ("COrder");
 *   HB_PLAN_SELECTIVE    ranked most selective (lowest sp) first ("SOrder");
 *   HB_PLAN_RANDOM_PREDS the heuristic path with each rule's predicates in a
 *                        random order ("noPO");
 *   HB_PLAN_RANDOM_RULES the heuristic path with the rules in a random order
 *                        ("noRO").
 * The random orders are drawn from a fixed seed (splitmix64 of the rule
 * set's first predicate ids), so repeated calls evaluate identically. */
typedef enum {
    HB_PLAN_GIVEN = 0,
    HB_PLAN_HEURISTIC = 1,
    HB_PLAN_LEARNED = 2,
    HB_PLAN_CHEAPEST = 3,
    HB_PLAN_SELECTIVE = 4,
    HB_PLAN_RANDOM_PREDS = 5,
    HB_PLAN_RANDOM_RULES = 6
} hb_plan;

/* Evaluate the rule set on every candidate pair and return Ca(D): packed
 * uint64 (i << 32) | j with i < j, sorted ascending, each pair once.  For
 * an ordered rule set (see the predicates), every ordered pair (i, j),
 * i != j, whose valuation t -> row i, s -> row j has a witness, sorted
 * ascending; each candidate pair is still visited once, its symmetric
 * predicates evaluated once for both orders.  Ordered rule sets take the
 * given, heuristic and strategy plans; HB_PLAN_LEARNED, hb_match_work,
 * hb_log_collect and batches reject them (HB_ERR_INVALID_ARG).
 * `out_pairs` holds `capacity` entries in host memory (out_on_device = 0)
 * or device memory (1).  If capacity is too small the call returns
 * HB_ERR_CAPACITY with *n_pairs = the size needed; the result stays cached
 * so a retry with a larger buffer only copies.  Requires hb_partition. */
hb_status hb_match(hb_ctx* ctx, uint32_t rel_id, uint32_t ruleset_id, int32_t plan,
                   uint64_t* out_pairs, int out_on_device, uint64_t capacity, uint64_t* n_pairs);

/* hb_match for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.  It
 * allocates nothing (no hipMalloc, no hipFree, no call of the context's
 * allocator): every device buffer of the call (block-major feature
 * columns, plan code, the unsorted pairs, the sort's histograms) is carved
 * from a scratch array of HB_NOALLOC_SCRATCH_BYTES that the library holds
 * on each device it runs on until the process ends; its address is taken
 * once per device by hb_create.  Every plan but HB_PLAN_LEARNED (its
 * per-block plans need buffers of their own: HB_ERR_INVALID_ARG); the
 * result equals hb_match's.  `out_pairs` is DEVICE memory of `capacity`
 * entries; it also serves as the sort's second buffer, so its contents
 * beyond the result are undefined.  *n_pairs = the pairs found; capacity
 * below that: HB_ERR_CAPACITY (nothing is cached: a retry evaluates
 * again).  A call whose buffers do not fit the array (about 2M tuples of
 * six attributes) returns HB_ERR_LIMIT.  Calls on one device share its
 * array: calls that overlap in time on one device race (the array keeps
 * the last call's contents; each call clears what must start at zero).
 * Requires hb_partition; q-gram indexes and character signatures are built
 * by hb_compile_rules. */
#define HB_NOALLOC_SCRATCH_BYTES (256u << 20)
hb_status hb_match_noalloc(hb_ctx* ctx, uint32_t rel_id, uint32_t ruleset_id, int32_t plan,
                           uint64_t* out_pairs, uint64_t capacity, uint64_t* n_pairs);

/* Launch shape of hb_match and hb_match_noalloc on this context: the i-rows
 * a wave evaluates per batch against its 64 j-lanes, 16 (four batches per
 * 64 x 64 tile), 32 (two) or 64 (one; the default).  Larger batches pay each
 * plan step's fixed cost once for more pairs; the result is the same.  Ordered
 * rule sets and batches keep 16; hb_match_work follows the setting.  Other
 * values: HB_ERR_INVALID_ARG. */
hb_status hb_set_rows_per_wave(hb_ctx* ctx, uint32_t rows);

/* Second launch-shape setting of this context: a filter step of a wave
 * batch runs per lane (each lane evaluates only its own live rows, one per
 * round) when no lane has more than `max_rows` live rows and `max_rows` is
 * at most half the batch's rows; otherwise it runs for every row of the
 * batch.  0 (the default) takes the tuned threshold of the batch size.
 * Applies to every match launch of the context; the result is the same.
 * Values above 32: HB_ERR_INVALID_ARG. */
hb_status hb_set_sparse_rows(hb_ctx* ctx, uint32_t max_rows);

/* Work decomposition of the key partitions hb_partition builds after this
 * call: with `on`, consecutive blocks of at most 32 rows are packed into
 * windows of at most 64 positions, one 64 x 64 tile each, every pair masked
 * to its own block (instead of one tile per block), where such blocks are
 * at least a quarter of the partition's tiles.  The windows are built on
 * the host from the block table (one read-back per partition).  Off by
 * default: on the 5M long-title workload, whose blocks all hold at most 18
 * rows, it cut the match kernel by 3% but the window build cost more than
 * that.  The result is the same either way. */
hb_status hb_set_pack_small_blocks(hb_ctx* ctx, int on);

/* HB_PLAN_LEARNED keeps a key partition's per-block plans only when the
 * cost model predicts they save at least `min_saving` of the partition's
 * cost under the heuristic plan (default 0.25: distinct plans miss the
 * scalar cache that one shared plan hits, and smaller predicted savings did
 * not hold up in measurement); 0 keeps every per-block plan.  Values
 * outside [0, 1): HB_ERR_INVALID_ARG. */
hb_status hb_set_learned_min_saving(hb_ctx* ctx, float min_saving);

/* Where hb_compile_rules takes each distinct predicate's cost (the
 * denominator of the cost-effectiveness order, Section 4.2, "Predicate
 * ordering"):
 *   HB_COST_STATIC (default): per-operator formulas of the attribute's mean
 *     length;
 *   HB_COST_PAIR_NET: the paper's estimated cost (Section 4.2, "Estimated
 *     cost"): the per-pair model (HB_MODEL_PAIR) estimates the time of
 *     checking the predicate on each of `samples` sampled pairs of D x D
 *     (the sample of hb_pair_log_collect with `seed`, the same pairs for
 *     every predicate); a predicate's cost is the sum of its estimates,
 *     2^(16 * clamp(y, 0, 4)) - 1 cycles per pair for the model's second
 *     output y (NaN counts as 0), divided by the largest predicate's sum
 *     (each kept at or above 2^-20 of it; every cost 1 when all sums are
 *     zero or the relation has fewer than two tuples).  Compile then needs a
 *     trained per-pair model (HB_ERR_STATE), predicates that compare one
 *     attribute of both tuples (HB_ERR_INVALID_ARG otherwise) and at most 64
 *     distinct predicates (HB_ERR_LIMIT); it reads the sums back with one
 *     synchronisation.
 * Costs order predicates only: every plan's result is unchanged.  Samples
 * outside [1, 65536] or another source: HB_ERR_INVALID_ARG. */
#define HB_COST_STATIC 0
#define HB_COST_PAIR_NET 1
hb_status hb_set_cost_estimate(hb_ctx* ctx, int source, uint32_t samples, uint64_t seed);

/* ------------------------------------------------------------ introspection */

/* Per distinct predicate of a rule set (in first-appearance order): its
 * selectivity estimate sp in [0, 1] and normalised cost in (0, 1].
 * *n receives the number of distinct predicates; up to `cap` are written. */
hb_status hb_ruleset_estimates(hb_ctx* ctx, uint32_t ruleset_id, double* sp, double* cost,
                               uint32_t cap, uint32_t* n);

/* LSH bucket counts (1024 buckets) behind sp of distinct predicate `pred`. */
hb_status hb_ruleset_buckets(hb_ctx* ctx, uint32_t ruleset_id, uint32_t pred, uint64_t* counts,
                             uint64_t* n_valid);

/* Pure host: the sequential execution path of Section 4.2 / 5.1 for given
 * estimates.  Predicates are ids 0..n_preds-1; rule r lists rule_len[r] ids
 * starting at rule_preds[sum of earlier lengths].  Writes the rule order to
 * out_rules[n_rules] and, per rule in that order, its distinct predicates
 * in evaluation order to out_preds (at most the total input length);
 * *out_len receives the number written to out_preds. */
hb_status hb_epg_path(uint32_t n_preds, const double* sp, const double* cost, uint32_t n_rules,
                      const uint32_t* rule_len, const uint32_t* rule_preds, uint32_t* out_rules,
                      uint32_t* out_preds, uint32_t* out_len);

/* Pure host: as hb_epg_path, for any plan but HB_PLAN_LEARNED (which is
 * chosen per block on the device): the path hb_match evaluates for a rule
 * set with these estimates.  HB_ERR_INVALID_ARG for an unknown plan. */
hb_status hb_plan_path(uint32_t plan, uint32_t n_preds, const double* sp, const double* cost, uint32_t n_rules,
                       const uint32_t* rule_len, const uint32_t* rule_preds, uint32_t* out_rules,
                       uint32_t* out_preds, uint32_t* out_len);

/* Kernel timing: when enabled, HIP events bracket each kernel launch of the
 * named step on the context stream.  Names: "match", "partition_sort",
 * "gram_slots", "gram_build" (the q-gram codes and signatures), "char_sig",
 * "lsh", "gather", "output_sort", "log", "block_features", "plan_choice",
 * "pair_cost" (the per-pair network's estimate inside hb_compile_rules);
 * and, as host wall
 * time including synchronisation, "learned_plan" (building one key
 * partition's per-block learned plans) and "predict" (cost-model inference
 * inside it). */
hb_status hb_profile_enable(hb_ctx* ctx, int on);
hb_status hb_profile_query(hb_ctx* ctx, const char* name, double* total_ms, uint64_t* launches);
/* Algorithmic HBM bytes of the timed launches counted under `name` since
 * the last reset: what each launch must read once and write once (for
 * "match": its feature columns; for the streaming steps "gram_slots",
 * "gram_build", "char_sig", "lsh", "partition_sort",
 * "gather", "output_sort": their inputs and outputs), so bytes / time is
 * the step's effective bandwidth. */
hb_status hb_profile_bytes(hb_ctx* ctx, const char* name, double* bytes);
hb_status hb_profile_reset(hb_ctx* ctx);

/* Work counters of one instrumented evaluation pass: the same kernels with
 * counting compiled in (output-neutral and slower; for profiling only).  Per
 * plan operation kind (index: 0 value equality, 1 |a-b| <= d, 2 string
 * equality filter, 3 edit-distance filter, 4 Jaccard filter, 5 string
 * equality, 6 edit distance, 7 Jaccard): `waves` = the times a wave ran it
 * for its batch of 16 rows x 64 lanes, `lanes` = the pairs that evaluated
 * it, `passed` = the pairs for which it held, `work` = its work units (edit
 * distance: text bytes x 32-bit pattern words run; Jaccard: merged list
 * elements; string equality: bytes compared; kinds 0-4: the rounds a wave
 * ran it in the per-lane form, one live row per lane and round, taken when
 * no lane had more than four live rows; `waves` does not count those
 * steps).  A wave batch holds the context's rows per wave (16, 32 or 64).  `pairs` is
 * the number of candidate pairs evaluated.  `lane_ops` is the algorithmic
 * int32 lane-operations of the pairs evaluated: value equality 2, |a-b| <= d
 * 4, each exact filter 4, string equality 2 + 1 per byte, edit distance 17
 * per work unit (Myers), Jaccard 3 per merged element.  `issued_ops` is the
 * same count with what the kernel issues per operation (12 for each
 * signature filter, 1 for value equality, 3 for the string-equality
 * filter), and `batch_ops` that issued count charged for every lane of
 * every batch a cheap step ran on (the SIMD work the plan causes).
 * Requires hb_partition; leaves the cached hb_match result untouched. */
#define HB_N_OPKINDS 8
typedef struct {
    uint64_t pairs;
    uint64_t matched;
    uint64_t launches;
    uint64_t waves[HB_N_OPKINDS];
    uint64_t lanes[HB_N_OPKINDS];
    uint64_t passed[HB_N_OPKINDS];
    uint64_t work[HB_N_OPKINDS];
    double lane_ops;
    double batch_ops;
    double issued_ops;
} hb_work_stats;
hb_status hb_match_work(hb_ctx* ctx, uint32_t rel_id, uint32_t ruleset_id, int32_t plan, hb_work_stats* out);

/* ------------------------------------------------------------ cost model
 * The learned cost models: MLPs 16 -> 64 -> 64 -> 2 (ReLU after both
 * hidden layers, linear output).  The block model predicts (pass rate,
 * cost) of a predicate on a block from 16 block features, the per-block form
 * of the paper's shallow network trained on logs (Section 4.2, "Shallow
 * NNs", "Estimated cost"); the per-pair model (HB_MODEL_PAIR below) is that
 * network's per-pair form, predicting (satisfied, time of the check) of a
 * predicate on one pair.
 * Parameters: HB_MLP_PARAMS fp32 values, row-major, in the order W1 [16x64],
 * b1 [64], W2 [64x64], b2 [64], W3 [64x2], b3 [2], used as y = x W + b.
 * GEMMs round both operands to bf16 (nearest, ties to even) and accumulate
 * in fp32; bias, ReLU, the loss and Adam (beta1 0.9, beta2 0.999, eps 1e-8)
 * run in fp32.  The models belong to the context. */
#define HB_MLP_PARAMS 5378
#define HB_MLP_FEATURES 16
/* The context holds two models of this shape: the block model (the learned
 * plan's, trained on hb_log_collect rows) and the per-pair model (the
 * paper's network N of Section 4.2, trained on hb_pair_log_collect rows,
 * which HB_COST_PAIR_NET reads).  The hb_costmodel_* calls below act on the
 * selected one (the block model until this is called; HB_ERR_INVALID_ARG
 * for another value).  The learned plan always reads the block model. */
#define HB_MODEL_BLOCK 0
#define HB_MODEL_PAIR 1
hb_status hb_costmodel_select(hb_ctx* ctx, int which);
/* He-uniform weights from a splitmix64 stream of `seed`, zero biases. */
hb_status hb_costmodel_init(hb_ctx* ctx, uint64_t seed);
/* Copy parameters in / out (host arrays of n = HB_MLP_PARAMS floats);
 * setting them resets the Adam moments. */
hb_status hb_costmodel_set_params(hb_ctx* ctx, const float* params, uint32_t n);
hb_status hb_costmodel_get_params(hb_ctx* ctx, float* params, uint32_t n);
/* Minimise the mean squared error over rows x [n x 16] -> t [n x 2] with
 * Adam, `epochs` passes of mini-batches of `batch` rows in the given order.
 * Buffers are host (on_device = 0) or device memory.  *final_loss = mean
 * squared error accumulated over the last epoch. */
hb_status hb_costmodel_train(hb_ctx* ctx, const float* x, const float* t, uint64_t n_rows, int on_device,
                             uint32_t epochs, uint32_t batch, float lr, float* final_loss);
/* y [n x 2] = model(x [n x 16]). */
hb_status hb_costmodel_predict(hb_ctx* ctx, const float* x, uint64_t n_rows, int on_device, float* y,
                               int y_on_device);
/* For checking the kernels: one forward and backward pass on host rows,
 * writing to `out` (host) the concatenation Z1, H1, Z2, H2 [n x 64 each],
 * Y, dY [n x 2 each], dZ2, dZ1 [n x 64 each] (Z = pre-activation, H =
 * ReLU(Z), dY = d loss / d Y, dZ = d loss / d Z) and the HB_MLP_PARAMS
 * gradients, in parameter order.  out_len >= n (6 * 64 + 4) + HB_MLP_PARAMS. */
hb_status hb_costmodel_trace(hb_ctx* ctx, const float* x, const float* t, uint32_t n_rows, float* out,
                             uint64_t out_len);
/* One Adam step with the given host gradients (HB_MLP_PARAMS floats). */
hb_status hb_costmodel_adam_step(hb_ctx* ctx, const float* grads, float lr);
/* Persist the context's model and read it back, so a model trained on the
 * logs of earlier runs plans later ones (the paper trains its estimator
 * offline on historical logs, Section 4.2, "Shallow NNs").  File layout,
 * little-endian: the 8 bytes "HBCMODEL"; uint32 version (1); uint32 inputs,
 * hidden width, outputs and parameter count (16, 64, 2, HB_MLP_PARAMS);
 * uint32 model (HB_MODEL_BLOCK or HB_MODEL_PAIR: the selected model when
 * saved; loading needs the same selection); HB_MLP_PARAMS fp32 parameters in
 * the order above; uint64 FNV-1a
 * 64 hash of those parameter bytes.  hb_costmodel_save needs a model
 * (HB_ERR_STATE) and writes `path` whole or not at all (a temporary file
 * renamed over it); hb_costmodel_load checks every field, the size and the
 * hash (HB_ERR_INVALID_ARG on any mismatch or I/O failure, leaving the
 * context's model unchanged) and resets the Adam moments, as
 * hb_costmodel_set_params does.  `path` is a NUL-terminated file name. */
hb_status hb_costmodel_save(hb_ctx* ctx, const char* path);
hb_status hb_costmodel_load(hb_ctx* ctx, const char* path);

/* Logging pass for the cost model (the paper trains its estimator on
 * historical logs, Section 4.2): for every block (of every key partition,
 * in key order, blocks in ascending key value) and every distinct predicate
 * evaluated there (ascending id; the partition's own key equality is
 * implied and skipped), one row of HB_MLP_FEATURES block features and two
 * labels from `samples` waves of 64 sampled pairs, each pair evaluated on
 * every predicate without short-circuit: label 0 = fraction of sampled pairs
 * passing the predicate's first plan step (its exact necessary-condition
 * filter; for value predicates the predicate itself), label 1 =
 * log2(1 + clock cycles per wave evaluation of the whole predicate) / 16.
 * Sampled pairs of wave s of block b (positions inside the block, rows in
 * ascending row order): c = (seed ^ (key index << 56)) + ((b * samples + s)
 * << 7); i = h(c + 64) mod n_b; j_l = h(c + l) mod n_b for lane l, replaced
 * by (i + 1) mod n_b when equal to i; h = the splitmix64 output function.
 * Outputs (host, any may be NULL): features [cap x 16], labels [cap x 2],
 * meta [cap x 3] = (key index, block, predicate id), counts [cap x 4] =
 * (pairs sampled, pairs satisfying, cycles, pairs passing the first step).  If cap_rows is too small the
 * call returns HB_ERR_CAPACITY with *n_rows = rows needed. */
hb_status hb_log_collect(hb_ctx* ctx, uint32_t rel_id, uint32_t ruleset_id, uint32_t samples, uint64_t seed,
                         float* features, float* labels, uint32_t* meta, uint64_t* counts, uint64_t cap_rows,
                         uint64_t* n_rows);

/* Logging pass for the per-pair model (Section 4.2, "Evaluation cost":
 * T_p(t1, t2) is the time of checking predicate p on the pair): for every
 * distinct predicate (ascending id; each must compare one attribute of both
 * tuples, HB_ERR_INVALID_ARG otherwise; at most 64, HB_ERR_LIMIT) and every
 * sampled pair s of D x D,
 * one row: i = h(seed + 2s) mod n, j = h(seed + 2s + 1) mod n, j replaced by
 * (i + 1) mod n when equal to i (h = the splitmix64 output function;
 * needs no hb_partition).  Row x * samples + s holds
 *   features: 16 inputs -- one-hot kind (value equality, |a-b| <= d, string
 *     equality, edit distance, Jaccard), t1.A and t2.A present, byte lengths
 *     L1 / 64 and L2 / 64, then [L1 == L2] (string equality), pattern words
 *     of L1 / 4 and k / 16 (edit distance: words 0 up to 32 bytes, else
 *     ceil(L1 / 64)), or q-gram counts C1 / 64 and C2 / 64 (Jaccard), a flag
 *     for a Jaccard value shorter than q, Jaccard's num / den (fp32),
 *     min(L1, L2) / 64, |L1 - L2| / 64 and 1; a missing value has length
 *     and count 0;
 *   labels: 1 if the pair satisfies the predicate, else 0; and
 *     log2(1 + clock cycles) / 16 of one wave checking that pair exactly
 *     (every lane on the same pair; the check runs twice and the second,
 *     with the pair's values in the caches, is timed, less the cycles of an
 *     empty interval between two clock reads, floored at 0).
 * pairs [samples x 2] = (i, j).  Outputs are host arrays (any may be NULL).
 * samples in [1, 65536] (HB_ERR_INVALID_ARG otherwise); a relation with
 * fewer than two tuples gives no rows.  If cap_rows is too small the call
 * returns HB_ERR_CAPACITY with *n_rows = rows needed. */
hb_status hb_pair_log_collect(hb_ctx* ctx, uint32_t rel_id, uint32_t ruleset_id, uint32_t samples, uint64_t seed,
                              float* features, float* labels, uint32_t* pairs, uint64_t cap_rows,
                              uint64_t* n_rows);

/* Counters of the last hb_match: candidate pairs, pairs matched, launches
 * and tiles of the match kernel. */
typedef struct {
    uint64_t candidate_pairs;
    uint64_t matched_pairs;
    uint64_t tiles;
    uint64_t launches;
    uint64_t learned_blocks;   /* HB_PLAN_LEARNED: blocks running a learned plan */
    uint64_t fallback_blocks;  /* HB_PLAN_LEARNED: blocks kept on the heuristic plan */
    uint64_t learned_plans;    /* HB_PLAN_LEARNED: distinct per-block plans written */
    /* HB_PLAN_LEARNED: the cost model's predicted cost (abstract units) of the
     * blocks that may take a per-block plan, under the heuristic plan and
     * under the plans it chose, summed over key partitions.  A partition
     * whose predicted saving is under the context's minimum
     * (hb_set_learned_min_saving) runs the heuristic plan throughout
     * (its blocks count as fallback). */
    double predicted_heuristic;
    double predicted_chosen;
} hb_match_stats;
hb_status hb_last_match_stats(hb_ctx* ctx, hb_match_stats* out);

/* ------------------------------------------------------------ batches
 * Many (relation, rule set) jobs matched together (the paper's pipeline
 * batches its work for the device, Section 5): every job's key partitions
 * form one queue of 64 x 64 tiles (heaviest partitions first) that runs in
 * one of three launch forms -- each partition's match launch on four
 * concurrent streams (0), one workgroup per 16-row batch of a tile over the
 * whole queue (1), or a persistent grid whose workgroups take batches from
 * a global cursor (2) -- optionally captured in a HIP graph, so uneven jobs
 * share the device.  Every job must have run hb_partition; its relation
 * and rule set must stay loaded while the batch exists (HB_ERR_STALE_ID on
 * hb_batch_run otherwise).  Results equal hb_match's in every form. */
#define HB_MAX_BATCH_JOBS 4096
#define HB_BATCH_GRAPH 1u     /* capture the batch's launches in a HIP graph, replayed by hb_batch_run */
#define HB_BATCH_AUTOTUNE 2u  /* time the launch forms (hb_batch_info.form; the persistent grid at each
                                 work-grab size and occupancy) on the batch's first items; keep the fastest.
                                 Batches created without it (or a forced form) use the context's last tuned
                                 form (else form 0) */
/* Force a launch form (not with HB_BATCH_AUTOTUNE; HB_ERR_INVALID_ARG otherwise).  The persistent form
 * takes one batch per grab at the occupancy the LDS footprint allows; the one-workgroup-per-batch form
 * needs at most 2^30 - 8 tiles in the queue (HB_ERR_LIMIT otherwise). */
#define HB_BATCH_FORM_STREAMS 0x100u
#define HB_BATCH_FORM_MULTI 0x200u
#define HB_BATCH_FORM_PERSISTENT 0x300u
#define HB_BATCH_FORM_MASK 0x300u

typedef struct {
    uint32_t rel_id;
    uint32_t ruleset_id;
} hb_job;

/* Builds every job's partition plans (plan: hb_plan) and the work queue;
 * flags: HB_BATCH_*.  *batch_id receives the handle. */
hb_status hb_batch_create(hb_ctx* ctx, const hb_job* jobs, uint32_t n_jobs, int32_t plan, uint32_t flags,
                          uint32_t* batch_id);
/* Matches every job (replaying the graph if captured) and sorts each job's
 * pairs; *n_pairs_total (may be NULL) receives the sum over jobs. */
hb_status hb_batch_run(hb_ctx* ctx, uint32_t batch_id, uint64_t* n_pairs_total);
/* Job `job`'s Ca(D) of the last hb_batch_run, as hb_match returns it
 * (sorted packed pairs; capacity protocol as hb_match). */
hb_status hb_batch_result(hb_ctx* ctx, uint32_t batch_id, uint32_t job, uint64_t* out_pairs, int out_on_device,
                          uint64_t capacity, uint64_t* n_pairs);

typedef struct {
    uint32_t n_jobs, n_partitions;
    uint64_t work_items;        /* 64 x 64 tiles in the queue */
    int32_t form;               /* 0: each partition's own launch on 4 concurrent streams;
                                   1: one one-wave workgroup per 16-row batch of a tile over the whole queue;
                                   2: persistent grid (grid workgroups taking grab batches per atomic) */
    uint32_t grid, grab, occupancy, lds_bytes;
    int32_t graph;              /* 1 if captured */
    uint32_t n_tuned;           /* candidates timed by HB_BATCH_AUTOTUNE */
    double tune_ms[32];         /* their times on the sample, in (occupancy, grab) order */
    uint64_t fallback_blocks;   /* learned plan: blocks kept on the heuristic plan for structural reasons */
} hb_batch_info;
hb_status hb_batch_info_get(hb_ctx* ctx, uint32_t batch_id, hb_batch_info* info);
hb_status hb_batch_destroy(hb_ctx* ctx, uint32_t batch_id);

#ifdef __cplusplus
}
#endif
#endif /* HB_H */
