// The pair-evaluation kernel of libhb (gfx950).
//
// Work unit: a 16-row batch of a 64 x 64 tile (i-tile, j-tile) of the upper
// triangle of one block of a key partition, run by a one-wave workgroup
// (four per tile).  The batch's 16 tuples t_i are uniform across the wave:
// their feature columns (values, lengths, set sizes, signatures) and the
// plan are read with scalar loads; each of the 64 lanes holds one candidate
// t_j and reads its features from the same columns.  A lane keeps 16-bit
// masks (bit r: the pair (row r, its t_j)) of the pairs still alive in the
// current rule and of those already matched.
//
// The wave walks the sequential execution path (Section 5.1) for its 1,024
// pairs: steps in plan order, a rule-end checkpoint that records witnesses
// (Section 2, "Blocking"), and a wave-uniform jump to the checkpoint once no
// pair of the batch can still satisfy the current rule.  Within a rule the
// plan runs exact, cheap necessary-condition filters first (value
// predicates, length and character-signature bounds for edit distance, the
// q-gram signature bound for Jaccard), one vector instruction sequence per
// row appending the row's result bit with an add-with-carry; the expensive
// predicates (edit distance, Jaccard, string equality) then run row by row
// only where some lane passed every filter of the rule.  Once few pairs
// are left, a filter step runs per lane, one live row per round, instead
// of over the 16 rows.  Consecutive rules that start with the same cheap
// step share it (a guard step, run once); predicates shared further down
// are evaluated again in each rule (a cache cost more registers than it
// saved).  Matched lanes are compacted with a ballot, one atomic per
// wave-row.
//
// Edit distance: Myers' bit-parallel algorithm in Hyyro's formulation for
// the Levenshtein distance (pattern = t_i, one bit per pattern byte, the
// pattern-match table built once per row in the wave's LDS), 32-bit words
// for patterns <= 32 bytes, 64-bit words with carry chains up to 256 bytes.
// Jaccard: merge intersection of the sorted distinct q-gram codes.
#include <type_traits>

#include "hb_internal.h"

namespace hb {

namespace {

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// --------------------------------------------------------------- Myers

template <typename T, int W>
__device__ inline int myers(const T* __restrict__ peq, int m, const uint8_t* __restrict__ text, int n) {
    constexpr int B = sizeof(T) * 8;
    T Pv[W], Mv[W];
#pragma unroll
    for (int w = 0; w < W; ++w) { Pv[w] = ~(T)0; Mv[w] = 0; }
    int score = m;
    const T hb = (T)1 << ((m - 1) % B);
    // text bytes in batches of four independent loads
    uint32_t ch[4];
    for (int pos = 0; pos < n; ++pos) {
        if ((pos & 3) == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) ch[k] = pos + k < n ? text[pos + k] : 0u;
        }
        const T* eq = peq + ch[pos & 3] * W;
        T carry = 0, ph_in = 1, mh_in = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const T Eq = eq[w];
            const T pv = Pv[w], mv = Mv[w];
            const T Xv = Eq | mv;
            const T a = Eq & pv;
            const T sum = a + pv;
            const T c1 = sum < a ? 1 : 0;
            const T sum2 = sum + carry;
            const T c2 = sum2 < sum ? 1 : 0;
            carry = c1 | c2;
            const T Xh = (sum2 ^ pv) | Eq;
            T Ph = mv | ~(Xh | pv);
            T Mh = pv & Xh;
            if (w == W - 1) {
                score += (Ph & hb) ? 1 : 0;
                score -= (Mh & hb) ? 1 : 0;
            }
            const T ph_out = Ph >> (B - 1), mh_out = Mh >> (B - 1);
            Ph = (Ph << 1) | ph_in;
            Mh = (Mh << 1) | mh_in;
            ph_in = ph_out;
            mh_in = mh_out;
            Pv[w] = Mh | ~(Xv | Ph);
            Mv[w] = Ph & Xv;
        }
    }
    return score;
}

// Patterns longer than 64 bytes: the same recurrence over W words whose
// vertical delta vectors live in the wave's LDS (slot w * 64 + lane), so the
// rare long patterns do not cost registers on the common path.
__device__ inline int myers_long(const uint64_t* __restrict__ peq, int W, int m, const uint8_t* __restrict__ text,
                                 int n, uint64_t* st, int lane) {
    uint64_t* Pv = st;
    uint64_t* Mv = st + kMaxEdWords * 64;
    for (int w = 0; w < W; ++w) { Pv[w * 64 + lane] = ~0ull; Mv[w * 64 + lane] = 0; }
    int score = m;
    const uint64_t hb = 1ull << ((m - 1) & 63);
    uint32_t ch[4];
    for (int pos = 0; pos < n; ++pos) {
        if ((pos & 3) == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) ch[k] = pos + k < n ? text[pos + k] : 0u;
        }
        const uint64_t* eq = peq + ch[pos & 3] * W;
        uint64_t carry = 0, ph_in = 1, mh_in = 0;
        for (int w = 0; w < W; ++w) {
            const uint64_t Eq = eq[w];
            const uint64_t pv = Pv[w * 64 + lane], mv = Mv[w * 64 + lane];
            const uint64_t Xv = Eq | mv;
            const uint64_t a = Eq & pv;
            const uint64_t sum = a + pv;
            const uint64_t c1 = sum < a ? 1 : 0;
            const uint64_t sum2 = sum + carry;
            const uint64_t c2 = sum2 < sum ? 1 : 0;
            carry = c1 | c2;
            const uint64_t Xh = (sum2 ^ pv) | Eq;
            uint64_t Ph = mv | ~(Xh | pv);
            uint64_t Mh = pv & Xh;
            if (w == W - 1) {
                score += (Ph & hb) ? 1 : 0;
                score -= (Mh & hb) ? 1 : 0;
            }
            const uint64_t ph_out = Ph >> 63, mh_out = Mh >> 63;
            Ph = (Ph << 1) | ph_in;
            Mh = (Mh << 1) | mh_in;
            ph_in = ph_out;
            mh_in = mh_out;
            Pv[w * 64 + lane] = Mh | ~(Xv | Ph);
            Mv[w * 64 + lane] = Ph & Xv;
        }
    }
    return score;
}

__device__ inline int myers_dispatch(const uint8_t* peq_bytes, int words, int m, const uint8_t* text, int n,
                                     uint64_t* st, int lane) {
    if (m == 0) return n;
    if (n == 0) return m;
    if (words == 0) return myers<uint32_t, 1>((const uint32_t*)peq_bytes, m, text, n);
    if (words == 1) return myers<uint64_t, 1>((const uint64_t*)peq_bytes, m, text, n);
    return myers_long((const uint64_t*)peq_bytes, words, m, text, n, st, lane);
}

// Pattern-match table of pattern p (length m) in the wave's LDS.
// words == 0: 32-bit table of 256 entries; else 256 x words 64-bit entries.
__device__ inline void build_peq(uint8_t* peq_bytes, int words, const uint8_t* __restrict__ p, int m, int lane) {
    if (words == 0) {
        uint32_t* t = (uint32_t*)peq_bytes;
        for (int x = lane; x < 256; x += 64) t[x] = 0;
        wave_sync();
        for (int k = lane; k < m; k += 64) atomicOr(&t[p[k]], 1u << k);
    } else {
        unsigned long long* t = (unsigned long long*)peq_bytes;
        for (int x = lane; x < 256 * words; x += 64) t[x] = 0;
        wave_sync();
        for (int k = lane; k < m; k += 64) atomicOr(&t[(uint32_t)p[k] * words + (k >> 6)], 1ull << (k & 63));
    }
    wave_sync();
}

// |A & B| for sorted distinct code lists; a short string's list is its
// single whole-string code, comparable only with another short string's.
// A (the wave's row) is in LDS; B streams from global memory eight codes
// per batch of independent loads, and a pointer into A advances
// monotonically (both lists ascend).
__device__ inline uint32_t intersect(const uint32_t* __restrict__ A, uint32_t ca, bool ashort,
                                     const uint32_t* __restrict__ B, uint32_t cb, bool bshort) {
    if (ashort || bshort) return (ashort && bshort && A[0] == B[0]) ? 1u : 0u;
    uint32_t ia = 0, I = 0;
    for (uint32_t ib = 0; ib < cb && ia < ca; ib += 8) {
        uint32_t y[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) y[k] = ib + k < cb ? B[ib + k] : 0u;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (ib + k < cb) {
                while (ia < ca && A[ia] < y[k]) ++ia;
                if (ia < ca && A[ia] == y[k]) { ++I; ++ia; }
            }
        }
    }
    return I;
}

__device__ inline bool absdiff_le(int64_t a, int64_t b, int64_t d) {
    const uint64_t diff = a >= b ? (uint64_t)a - (uint64_t)b : (uint64_t)b - (uint64_t)a;
    return diff <= (uint64_t)d;
}

// Pointers that live in device memory, stated to the compiler: pointers
// read out of a parameter block in memory are otherwise generic, and
// generic loads of wave-uniform addresses do not become scalar loads.
// (The host pass of the single-source build only needs the kernels' stubs.)
#if defined(__HIP_DEVICE_COMPILE__)
#define HB_GLOBAL __attribute__((address_space(1)))
#else
#define HB_GLOBAL
#endif
template <typename T>
__device__ __forceinline__ const HB_GLOBAL T* gmem(const T* p) {
    return (const HB_GLOBAL T*)p;
}

// keep * 2 + (this lane's bit of `lanes`): one add-with-carry that takes
// the lane mask of a comparison as its carry-in, so a 16-row batch builds
// its per-lane row bits at one vector instruction per row.
__device__ __forceinline__ uint32_t push_bit(uint32_t keep, uint64_t lanes) {
    uint32_t out;
    uint64_t carry;
    asm("v_addc_co_u32_e64 %0, %1, %2, %2, %3" : "=v"(out), "=s"(carry) : "v"(keep), "s"(lanes));
    return out;
}

// popcount(x) + acc in one instruction (the compiler otherwise sums the
// halves of a 64-bit popcount with a separate three-way add).
__device__ __forceinline__ uint32_t popc_add(uint32_t x, uint32_t acc) {
    uint32_t out;
    asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(out) : "v"(x), "v"(acc));
    return out;
}

// a * b + c on the signed 24-bit multiplier (|a|, |b| < 2^23), one
// full-rate instruction; the caller keeps the result within int32.
__device__ __forceinline__ int mad_i24(int a, int b, int c) {
    int out;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(out) : "v"(a), "s"(b), "v"(c));
    return out;
}

// Opaque copy: keeps the compiler from folding a precomputed per-lane term
// back into the per-row arithmetic.
template <typename T>
__device__ __forceinline__ T opaque(T v) {
    asm("" : "+v"(v));
    return v;
}

// Bit r (r < kR): bit `bit` of the validity word of position p0 + r.  All
// operands are wave-uniform, so this runs on the scalar unit.
// Row mask of a batch of kR rows (bit r: row r): 32 bits up to 32 rows,
// 64 beyond.
template <int kR>
using RowMask = typename std::conditional<(kR > 32), uint64_t, uint32_t>::type;

template <typename M>
__device__ __forceinline__ uint32_t popc_rows(M m) {
    if constexpr (sizeof(M) == 8) return (uint32_t)__popcll(m); else return (uint32_t)__popc(m);
}
template <typename M>
__device__ __forceinline__ uint32_t ctz_rows(M m) {
    if constexpr (sizeof(M) == 8) return (uint32_t)__builtin_ctzll(m); else return (uint32_t)__builtin_ctz(m);
}

// Builds a lane's row mask one row at a time, from the last row to the
// first, with push_bit (one add-with-carry per row); 64-row masks fill two
// 32-bit halves.  Row indices are compile-time in the unrolled loops, so
// the choice of half costs nothing.
template <int kR>
struct RowPush {
    uint32_t lo = 0, hi = 0;
    __device__ __forceinline__ void push(int r, uint64_t lanes) {
        if (kR > 32 && r >= 32) hi = push_bit(hi, lanes);
        else lo = push_bit(lo, lanes);
    }
    __device__ __forceinline__ RowMask<kR> get() const {
        if constexpr (kR > 32) return ((uint64_t)hi << 32) | lo; else return lo;
    }
};

template <int kR>
__device__ __forceinline__ RowMask<kR> row_bits(const HB_GLOBAL uint32_t* __restrict__ vmask, uint64_t p0,
                                                 uint32_t bit) {
    uint32_t lo = 0, hi = 0;
#pragma unroll
    for (int r = kR - 1; r >= 0; --r) {
        const uint32_t v = (vmask[p0 + r] >> bit) & 1u;
        if (kR > 32 && r >= 32) hi = hi + hi + v;
        else lo = lo + lo + v;
    }
    if constexpr (kR > 32) return ((uint64_t)hi << 32) | lo; else return lo;
}

// tile index -> (block, ti, tj), tiles of a block enumerated column-major
// over the upper triangle: column tj holds ti = 0..tj.
__device__ inline void decode_tile(const MatchParams& P, uint64_t t, uint32_t* b, uint32_t* ti, uint32_t* tj) {
    const HB_GLOBAL uint64_t* tp = gmem(P.tile_prefix);
    const uint32_t lo = gmem(P.tile_blk)[t];
    *b = lo;
    const uint64_t u = t - tp[lo];
    uint64_t c = (uint64_t)((sqrt(8.0 * (double)u + 1.0) - 1.0) * 0.5);
    while (c * (c + 1) / 2 > u) --c;
    while ((c + 1) * (c + 2) / 2 <= u) ++c;
    *tj = (uint32_t)c;
    *ti = (uint32_t)(u - c * (c + 1) / 2);
}

// 16-row batch `batch` of the 64 x 64 tile t of partition P, by one wave:
// the batch's i-rows are wave-uniform (scalar loads), each lane holds one
// j-row and reads its features from the columns when a step needs them.
// Wave-uniform values are passed through readfirstlane so the compiler
// keeps them (and the loads they address) scalar.
// kOrd (rule sets that tell t from s): the pair (row r, lane j) has two
// valuations, t -> row, s -> lane ("forward") and t -> lane, s -> row
// ("backward"), each with its own alive and matched masks; symmetric steps
// run once for the union and narrow both, and each valuation that reaches
// a checkpoint emits its ordered pair.
template <bool kCount, bool kLongEd = false, bool kOrd = false, int kR = kRows>
__device__ __forceinline__ void match_tile(const MatchParams& P, const HB_GLOBAL Instr* __restrict__ plan,
                                           const HB_GLOBAL uint64_t* __restrict__ f64,
                                           const HB_GLOBAL uint32_t* __restrict__ f32, uint64_t t, uint8_t* lds,
                                           int batch) {
    using Mask = RowMask<kR>;
    constexpr Mask kAll = ~(Mask)0;
    const int lane = threadIdx.x & 63;
    const int wave = batch;
    uint32_t b, ti, tj;
    decode_tile(P, t, &b, &ti, &tj);
    // the tile's unit: a block, or a window of small blocks (one tile)
    uint32_t bstart, bsize;
    uint64_t bounds = 0;   // window: bit k set where position k ends its block
    bool packed = false;
    if (P.unit_start) {
        const uint32_t u = b, us = gmem(P.unit_size)[u];
        bstart = gmem(P.unit_start)[u];
        packed = (us & kPackedUnit) != 0;
        bsize = us & ~kPackedUnit;
        b = gmem(P.unit_blk)[u];   // the block (per-block plans), ~0u for a window
        if (packed) bounds = gmem(P.unit_bounds)[u];
    } else {
        bstart = gmem(P.blk_start)[b];
        bsize = gmem(P.blk_size)[b];
    }
    const uint32_t i0 = ti * kTile, j0 = tj * kTile;
    const uint32_t ni = min((uint32_t)kTile, bsize - i0), nj = min((uint32_t)kTile, bsize - j0);
    const bool diag = ti == tj;

    const uint64_t n = P.feat.n;
    const uint32_t str64 = P.n_int, gram64 = P.n_int + P.n_str;    // first f64 column of each kind
    const uint32_t str32 = 2, gram32 = 2 + P.n_str;                 // first f32 column of each kind
    const uint32_t jf32 = gram32 + P.n_gram;

    // j features of this lane: lanes past the block read the next
    // positions, which the column padding keeps in bounds, and their pairs
    // are masked off
    const uint64_t pj = (uint64_t)bstart + j0;
    auto J64 = [&](uint32_t col) -> uint64_t { return f64[col * n + pj + lane]; };
    auto J32 = [&](uint32_t col) -> uint32_t { return f32[col * n + pj + lane]; };
    unsigned long long* s_cnt = (unsigned long long*)(lds + P.lds_counts);
    if constexpr (kCount)
        for (uint32_t x = lane; x < kCountSlots; x += 64) s_cnt[x] = 0;
    __syncthreads();

    // this wave's rows: r0 .. r0 + nr - 1 of the i-tile (16 consecutive rows)
    const uint32_t r0 = (uint32_t)wave * kR;
    const int nr = (int)min((uint32_t)kR, ni > r0 ? ni - r0 : 0u);
    if (!kCount && nr <= 0) return;
    if (nr > 0) {
        const uint64_t pi0 = (uint64_t)bstart + i0 + r0;   // position of row 0
        const uint32_t row_j = J32(0);
        // validity: every row valid on every attribute the plan reads when
        // the relation has no missing values there (the mask words are then
        // not read)
        const bool all_valid = P.all_valid != 0;
        const uint32_t vmask_j = all_valid ? ~0u : J32(1);
        auto rvalid = [&](uint32_t bit) -> Mask { return all_valid ? kAll : row_bits<kR>(f32 + n, pi0, bit); };
        uint8_t* wbase = lds;
        uint8_t* peq = wbase + P.lds_wave_peq;
        const HB_GLOBAL Instr* __restrict__ pl = plan;
        uint32_t plen = P.plan_len;
        if (P.blk_slot && !packed) pl = plan + (size_t)gmem(P.blk_slot)[b] * plen;

        // bit r of a lane's masks = the pair (row r, this lane's j): lanes
        // below nj, and on a diagonal tile only j > i (lanes above r0 + r)
        const uint64_t lanes_j = nj >= 64 ? ~0ull : (1ull << nj) - 1ull;
        Mask pairs;
        if (!packed) {
            RowPush<kR> acc;
#pragma unroll
            for (int r = kR - 1; r >= 0; --r) {
                const uint32_t above = r0 + (uint32_t)r + 1u;
                const uint64_t upper = !diag ? ~0ull : above >= 64 ? 0ull : ~0ull << above;
                acc.push(r, r < nr ? lanes_j & upper : 0ull);
            }
            pairs = acc.get();
        } else {
            // a window (one diagonal tile): row k pairs with the lanes after
            // it up to its block's last position, the next set bit of bounds
            RowPush<kR> acc;
#pragma unroll
            for (int r = kR - 1; r >= 0; --r) {
                const uint32_t k = r0 + (uint32_t)r;
                const uint64_t rest = k < 64 ? bounds >> k : 0ull;
                const uint32_t end = rest ? k + 1u + (uint32_t)__builtin_ctzll(rest) : 0u;   // block end, exclusive
                const uint64_t upper = k + 1 >= 64 ? 0ull : ~0ull << (k + 1);
                const uint64_t below = end >= 64 ? ~0ull : (1ull << end) - 1ull;
                acc.push(r, r < nr ? lanes_j & upper & below : 0ull);
            }
            pairs = acc.get();
        }
        // canonical owner: a pair agreeing on an earlier key was evaluated there
        for (uint32_t k = 0; k < P.n_prev; ++k) {
            const uint32_t res = P.prev_res[k];
            const uint64_t vj = J64(res);
            RowPush<kR> acc;
#pragma unroll
            for (int r = kR - 1; r >= 0; --r) acc.push(r, __ballot(f64[res * n + pi0 + r] == vj));
            const Mask same = acc.get();
            pairs &= (vmask_j >> res) & 1 ? ~(same & rvalid(res)) : kAll;
        }
        if constexpr (kCount) {
            uint32_t cnt = 0;
            for (int r = 0; r < kR; ++r) cnt += __popcll(__ballot((pairs >> r) & 1));
            if (lane == 0 && cnt) atomicAdd(&s_cnt[kCountPairs], (unsigned long long)cnt);
        }

        // the per-lane form pays per-lane loads each round: taken when no
        // lane has more than min(4, rows / 2) live rows
        const uint32_t sparse_max = min(sparse_rows(P.sparse_rows, kR), (uint32_t)nr >> 1);
        Mask matched = 0, alive = pairs;
        Mask fwd = pairs, bwd = pairs, matched_b = 0;   // kOrd only: alive = fwd | bwd
        // the pairs a rule starts from: every pair, or inside a group of
        // rules those that passed the group's shared step (until its end)
        Mask base = pairs;
        uint32_t group_end = 0;
        bool in_group = false;
        uint32_t pc = 0;
        while (pc < plen) {
            pc = __builtin_amdgcn_readfirstlane(pc);
            // one 16-byte scalar load (there is no scalar byte load)
            const uint4 raw = *(const HB_GLOBAL uint4*)(pl + pc);
            // every word is needed before the step's own loads: one 16-byte
            // load and one wait, not a dependent load per field
            asm volatile("" ::"s"(raw.x), "s"(raw.y), "s"(raw.z), "s"(raw.w));
            uint32_t op = raw.x & 0xFFu;
            const uint32_t res = (raw.x >> 16) & 0xFFu;
            const uint32_t cp = raw.y & 0xFFFFu;
            const uint64_t param = ((uint64_t)raw.w << 32) | raw.z;
            if (op == OP_CP) {
                if constexpr (kOrd) {
                    matched |= fwd;
                    matched_b |= bwd;
                    fwd = pairs & ~matched;
                    bwd = pairs & ~matched_b;
                    alive = fwd | bwd;
                } else {
                    matched |= alive;
                    alive = base & ~matched;
                }
                if (!__any(alive != 0)) {
                    if (!in_group) break;   // every pair is matched or absent
                    pc = group_end;         // the group's rules have no pair left
                    continue;
                }
                ++pc;
                continue;
            }
            if (op == OP_ENDGUARD) {
                base = pairs;
                in_group = false;
                alive = pairs & ~matched;
                if (!__any(alive != 0)) break;
                ++pc;
                continue;
            }
            if (!__any(alive != 0)) { pc = cp; continue; }
            const bool guard = op == OP_GUARD;
            if (guard) op = (raw.x >> 24) & 0xFFu;   // the shared step's own operation
            if constexpr (kOrd) {
                if (op >= OP_CONST) {
                    // a predicate that tells t from s: one mask per valuation
                    const uint32_t aux = (raw.x >> 24) & 0xFFu;
                    Mask kf, kb;
                    if (op == OP_CONST) {   // t.A = c (aux 0) or s.A = c (aux 1), A = res
                        const int64_t c = (int64_t)param;
                        const Mask lane_hit = ((vmask_j >> res) & 1) && (int64_t)J64(res) == c ? kAll : (Mask)0;
                        RowPush<kR> acc;
#pragma unroll
                        for (int r = kR - 1; r >= 0; --r)
                            acc.push(r, __ballot((int64_t)f64[res * n + pi0 + (uint64_t)r] == c));
                        Mask rows = acc.get();
                        rows &= rvalid(res);
                        kf = aux == 0 ? rows : lane_hit;
                        kb = aux == 0 ? lane_hit : rows;
                    } else if (op == OP_XED) {
                        // Levenshtein(t.A, s.B) <= k, A = res, B = aux: forward
                        // runs the row's A against the lane's B, backward the
                        // row's B against the lane's A (the distance is
                        // symmetric in its strings), row by row where some
                        // lane needs it, the pattern table built from the row
                        const int k = (int)param;
                        kf = 0;
                        kb = 0;
                        for (int r = 0; r < nr; ++r) {
                            const uint64_t pi = pi0 + r;
                            const uint32_t row_i = f32[pi];
                            const uint32_t vmask_i = f32[n + pi];
#pragma unroll 1
                            for (int dir = 0; dir < 2; ++dir) {
                                const uint32_t pa = dir == 0 ? res : aux;   // row side (pattern)
                                const uint32_t ta = dir == 0 ? aux : res;   // lane side (text)
                                const bool need = (((dir == 0 ? fwd : bwd) >> r) & 1) &&
                                                  ((vmask_i >> (16 + pa)) & 1) && ((vmask_j >> (16 + ta)) & 1);
                                const int m = (int)f32[(str32 + pa) * n + pi];
                                const int nn = (int)J32(str32 + ta);
                                const bool run = need && abs(m - nn) <= k;
                                if (!__any(run)) continue;
                                const ColDev& col_p = P.cols[P.str_attr[pa]];
                                const ColDev& col_t = P.cols[P.str_attr[ta]];
                                const int words = m <= 32 ? 0 : (m + 63) / 64;
                                build_peq(peq, words, col_p.bytes + col_p.off[row_i], m, lane);
                                if (run) {
                                    const uint8_t* tj = col_t.bytes + col_t.off[row_j];
                                    int dist;
                                    if constexpr (kLongEd) {
                                        dist = m == 0 ? nn : nn == 0 ? m
                                             : words == 0 ? myers<uint32_t, 1>((const uint32_t*)peq, m, tj, nn)
                                             : words == 1 ? myers<uint64_t, 1>((const uint64_t*)peq, m, tj, nn)
                                             : words == 2 ? myers<uint64_t, 2>((const uint64_t*)peq, m, tj, nn)
                                             : words == 3 ? myers<uint64_t, 3>((const uint64_t*)peq, m, tj, nn)
                                                          : myers<uint64_t, 4>((const uint64_t*)peq, m, tj, nn);
                                    } else {
                                        dist = myers_dispatch(peq, words, m, tj, nn,
                                                              (uint64_t*)(wbase + P.lds_wave_myers), lane);
                                    }
                                    if (dist <= k) {
                                        if (dir == 0) kf |= (Mask)1 << r;
                                        else kb |= (Mask)1 << r;
                                    }
                                }
                            }
                        }
                    } else if (op == OP_XJAC || op == OP_XCONT) {
                        // Jaccard(G_q(t.A), G_q(s.B)) >= num / den, or the
                        // containment of G_q(t.A) in G_q(s.B) (asymmetric: the
                        // intersection over t's set), A = res, B = aux (gram
                        // resources of one q): forward merges the row's A list,
                        // staged in LDS, with the lane's B list, backward the
                        // row's B with the lane's A, row by row where some lane
                        // needs it
                        const bool cont = op == OP_XCONT;
                        const uint32_t num = (uint32_t)(param >> 32), den = (uint32_t)(param & 0xFFFFFFFFu);
                        kf = 0;
                        kb = 0;
                        for (int r = 0; r < nr; ++r) {
                            const uint64_t pi = pi0 + r;
                            const uint32_t row_i = f32[pi];
                            const uint32_t vmask_i = f32[n + pi];
#pragma unroll 1
                            for (int dir = 0; dir < 2; ++dir) {
                                const uint32_t ga = dir == 0 ? res : aux;   // row side
                                const uint32_t gb = dir == 0 ? aux : res;   // lane side
                                const bool need = (((dir == 0 ? fwd : bwd) >> r) & 1) &&
                                                  ((vmask_i >> (24 + ga)) & 1) && ((vmask_j >> (24 + gb)) & 1);
                                if (!__any(need)) continue;
                                const GramDev& g_a = P.gram[ga];
                                const GramDev& g_b = P.gram[gb];
                                const uint32_t ia = f32[(gram32 + ga) * n + pi];
                                const uint32_t ca = ia & 0x7FFFFFFFu;
                                uint32_t* ig = (uint32_t*)(wbase + P.lds_wave_igram[ga]);
                                const uint32_t* src = g_a.codes + g_a.off[row_i];
                                for (uint32_t x = lane; x < ca; x += 64) ig[x] = src[x];
                                wave_sync();
                                if (need) {
                                    const uint32_t jb = J32(gram32 + gb);
                                    const uint32_t cb = jb & 0x7FFFFFFFu;
                                    const uint32_t I = intersect(ig, ca, (ia >> 31) != 0, g_b.codes + g_b.off[row_j], cb,
                                                                 (jb >> 31) != 0);
                                    // the denominator: the union, or t's set (the row's
                                    // A forward, the lane's A backward)
                                    const uint64_t U = cont ? (dir == 0 ? ca : cb) : (uint64_t)ca + cb - I;
                                    if (U == 0 || (uint64_t)I * den >= (uint64_t)num * U) {
                                        if (dir == 0) kf |= (Mask)1 << r;
                                        else kb |= (Mask)1 << r;
                                    }
                                }
                                wave_sync();   // the staging area is refilled for the next list
                            }
                        }
                    } else {   // OP_XEQ: t.A = s.B, A = res, B = aux
                        const int64_t ja = (int64_t)J64(res), jb = (int64_t)J64(aux);
                        RowPush<kR> fa, ga;
#pragma unroll
                        for (int r = kR - 1; r >= 0; --r) {
                            const uint64_t pr = pi0 + (uint64_t)r;
                            fa.push(r, __ballot((int64_t)f64[res * n + pr] == jb));   // t = row: row.A = lane.B
                            ga.push(r, __ballot((int64_t)f64[aux * n + pr] == ja));   // t = lane: lane.A = row.B
                        }
                        const Mask f = fa.get(), g = ga.get();
                        kf = (vmask_j >> aux) & 1 ? f & rvalid(res) : (Mask)0;
                        kb = (vmask_j >> res) & 1 ? g & rvalid(aux) : (Mask)0;
                    }
                    fwd &= kf;
                    bwd &= kb;
                    alive = fwd | bwd;
                    ++pc;
                    continue;
                }
            }
            const Mask before = alive;
            uint32_t work = 0;
            // Few pairs left per lane (the usual state after a rule's first
            // filter): each lane evaluates only its own live pairs, one row
            // per round, reading that row's features with per-lane loads,
            // instead of the batch's 16 rows.  The arithmetic is the batch
            // form's, row for row.
            const bool single = op <= OP_JACF && !__any(popc_rows(alive) > sparse_max);
            if (single) {
                // one live row per lane and round; the operation's lane-side
                // operands are read once, the row's from its column with a
                // uniform base and a 32-bit lane offset.  A lane whose own
                // value is missing fails every row at once; a row's validity
                // bit `vbit` is read only where the relation has missing
                // values (kValid false).
                const uint32_t* vcol = f32 + n + pi0;   // the rows' validity words
                auto rounds = [&](auto valid_tag, bool lane_ok, uint32_t vbit, auto&& test) -> uint32_t {
                    constexpr bool kValid = decltype(valid_tag)::value;
                    Mask rem = lane_ok ? alive : (Mask)0, keep = 0;
                    uint32_t n_rounds = 0;
                    while (__any(rem != 0)) {
                        ++n_rounds;
                        const uint32_t r = rem != 0 ? ctz_rows(rem) : 0u;
                        // every load of the round issued together: no
                        // short-circuit between the conditions
                        bool ok = test(r);
                        if constexpr (!kValid) ok = ok & (((vcol[r] >> vbit) & 1) != 0);
                        if (rem != 0 && ok) keep |= (Mask)1 << r;
                        rem &= rem - 1;
                    }
                    alive = keep;
                    return n_rounds;
                };
                auto rounds_of = [&](bool lane_ok, uint32_t vbit, auto&& test) -> uint32_t {
                    return all_valid ? rounds(std::true_type{}, lane_ok, vbit, test)
                                     : rounds(std::false_type{}, lane_ok, vbit, test);
                };
                switch (op) {
                case OP_EQ_INT:
                case OP_ABSDIFF: {
                    const int64_t vj = (int64_t)J64(res);
                    const int64_t d = op == OP_EQ_INT ? 0 : (int64_t)param;
                    const int64_t lo = vj < INT64_MIN + d ? INT64_MIN : vj - d;
                    const int64_t hi = vj > INT64_MAX - d ? INT64_MAX : vj + d;
                    const int64_t* col = (const int64_t*)f64 + (uint64_t)res * n + pi0;
                    work = rounds_of((vmask_j >> res) & 1, res, [&](uint32_t r) {
                        const int64_t vi = col[r];
                        return (vi >= lo) & (vi <= hi);
                    });
                    break;
                }
                case OP_EQF: {
                    const uint32_t lj = J32(str32 + res);
                    const uint64_t cj = J64(str64 + res);
                    const uint32_t* lcol = f32 + (uint64_t)(str32 + res) * n + pi0;
                    const uint64_t* ccol = f64 + (uint64_t)(str64 + res) * n + pi0;
                    work = rounds_of((vmask_j >> (16 + res)) & 1, 16 + res, [&](uint32_t r) {
                        return (lcol[r] == lj) & (ccol[r] == cj);
                    });
                    break;
                }
                case OP_EDF: {
                    const int lj = (int)J32(str32 + res);
                    const uint64_t cj = J64(str64 + res);
                    const int k = (int)param;
                    const int tj = (int)__popcll(cj) - k;
                    const uint32_t* lcol = f32 + (uint64_t)(str32 + res) * n + pi0;
                    const uint64_t* ccol = f64 + (uint64_t)(str64 + res) * n + pi0;
                    work = rounds_of((vmask_j >> (16 + res)) & 1, 16 + res, [&](uint32_t r) {
                        const int li = (int)lcol[r];
                        const uint64_t ci = ccol[r];
                        const int both = (int)(__popc((uint32_t)ci & (uint32_t)cj) +
                                               __popc((uint32_t)(ci >> 32) & (uint32_t)(cj >> 32)));
                        const int t = max((int)__popcll(ci) - k, tj);
                        return (both >= t) & (li >= lj - k) & (li <= lj + k);
                    });
                    break;
                }
                default: {   // OP_JACF: the bound of the batch form, in exact 64-bit arithmetic
                    const uint32_t num = (uint32_t)(param >> 32), nd = num + (uint32_t)(param & 0xFFFFFFFFu);
                    if (num == 0) {   // every pair of present values
                        work = rounds_of((vmask_j >> (24 + res)) & 1, 24 + res, [](uint32_t) { return true; });
                        break;
                    }
                    // the filter words fail a missing value against anything
                    // (num > 0): no validity bit is read
                    const uint32_t gcol = gram64 + P.gram[res].sig_col;
                    const uint32_t wb = J32(jf32 + res);
                    const uint32_t* wcol = f32 + (uint64_t)(jf32 + res) * n + pi0;
                    const uint64_t* gcol0 = f64 + (uint64_t)gcol * n + pi0;
                    if (P.gram[res].sig_words == 1) {
                        const uint64_t gj = J64(gcol);
                        work = rounds(std::true_type{}, true, 0, [&](uint32_t r) {
                            const uint32_t wa = wcol[r];
                            const uint64_t gi = gcol0[r];
                            const uint32_t iub = min(wa >> 16, wb >> 16) + (uint32_t)__popcll(gi & gj);
                            return (uint64_t)iub * nd >= (uint64_t)num * ((wa & 0xFFFFu) + (wb & 0xFFFFu));
                        });
                    } else {   // the four-word signature of long strings
                        uint64_t gjw[kLongSigWords];
#pragma unroll
                        for (uint32_t w = 0; w < kLongSigWords; ++w) gjw[w] = J64(gcol + w);
                        work = rounds(std::true_type{}, true, 0, [&](uint32_t r) {
                            const uint32_t wa = wcol[r];
                            uint32_t iub = min(wa >> 16, wb >> 16);
#pragma unroll
                            for (uint32_t w = 0; w < kLongSigWords; ++w)
                                iub += (uint32_t)__popcll(gcol0[(uint64_t)w * n + r] & gjw[w]);
                            return (uint64_t)iub * nd >= (uint64_t)num * ((wa & 0xFFFFu) + (wb & 0xFFFFu));
                        });
                    }
                    break;
                }
                }
            } else switch (op) {
            case OP_EQ_INT:
            case OP_ABSDIFF: {
                const int64_t vj = (int64_t)J64(res);
                const uint32_t jv = (vmask_j >> res) & 1;
                // |vi - vj| <= d  <=>  vj - d <= vi <= vj + d, the ends
                // saturated to the int64 range (d >= 0; equality: d = 0)
                const int64_t d = op == OP_EQ_INT ? 0 : (int64_t)param;
                const int64_t lo = opaque(vj < INT64_MIN + d ? INT64_MIN : vj - d);
                const int64_t hi = opaque(vj > INT64_MAX - d ? INT64_MAX : vj + d);
                RowPush<kR> acc;
#pragma unroll
                for (int r = kR - 1; r >= 0; --r) {   // bit r of keep: row r
                    const uint64_t pr = pi0 + (uint64_t)r;   // rows >= nr: masked off, read in the pad
                    const int64_t vi = (int64_t)f64[res * n + pr];
                    acc.push(r, __ballot(vi >= lo) & __ballot(vi <= hi));
                }
                alive &= jv ? acc.get() & rvalid(res) : (Mask)0;
                work = 1;
                break;
            }
            case OP_EQF: {
                const uint32_t lj = J32(str32 + res);
                const uint64_t cj = J64(str64 + res);
                const uint32_t jv = (vmask_j >> (16 + res)) & 1;
                RowPush<kR> acc;
#pragma unroll
                for (int r = kR - 1; r >= 0; --r) {
                    const uint64_t pr = pi0 + (uint64_t)r;
                    const uint32_t li = f32[(str32 + res) * n + pr];
                    const uint64_t ci = f64[(str64 + res) * n + pr];
                    acc.push(r, __ballot(li == lj) & __ballot(ci == cj));
                }
                alive &= jv ? acc.get() & rvalid(16 + res) : (Mask)0;
                work = 1;
                break;
            }
            case OP_EDF: {
                // ED <= k needs |li - lj| <= k and, for the character
                // signatures, |ci \ cj| <= k and |cj \ ci| <= k, where
                // |ci \ cj| = |ci| - |ci & cj|: both hold iff
                // |ci & cj| >= max(|ci| - k, |cj| - k)
                const int lj = (int)J32(str32 + res);
                const uint64_t cj = J64(str64 + res);
                const uint32_t jv = (vmask_j >> (16 + res)) & 1;
                const int k = (int)param;
                const int llo = opaque(lj - k), lhi = opaque(lj + k);
                const int tj = opaque((int)__popcll(cj) - k);
                const uint32_t cj_lo = (uint32_t)cj, cj_hi = (uint32_t)(cj >> 32);
                RowPush<kR> acc;
#pragma unroll
                for (int r = kR - 1; r >= 0; --r) {
                    const uint64_t pr = pi0 + (uint64_t)r;
                    const int li = (int)f32[(str32 + res) * n + pr];
                    const uint64_t ci = f64[(str64 + res) * n + pr];
                    const int both = (int)(__popc((uint32_t)ci & cj_lo) + __popc((uint32_t)(ci >> 32) & cj_hi));
                    const int t = max((int)__popcll(ci) - k, tj);
                    acc.push(r, __ballot(both >= t) & __ballot(li >= llo) & __ballot(li <= lhi));
                }
                alive &= jv ? acc.get() & rvalid(16 + res) : (Mask)0;
                work = 1;
                break;
            }
            case OP_JACF: {
                // I <= |A| - |gA \ gB| and I <= |B| - |gB \ gA| with
                // |gA \ gB| = |gA| - |gA & gB|: the bound is
                // |gA & gB| + min(|A| - |gA|, |B| - |gB|), against
                // I * (num + den) >= num * (|A| + |B|).  Set sizes are
                // <= 4096 and den <= 2^18, so every product fits 32 bits
                // and takes the full-rate 24-bit multiplier.  The filter
                // words carry both sizes, and a missing value's word fails
                // against anything once num > 0.
                const uint32_t wb = J32(jf32 + res);
                const uint32_t gcol = gram64 + P.gram[res].sig_col;
                const uint64_t gj = J64(gcol);
                const uint32_t num = (uint32_t)(param >> 32), nd = num + (uint32_t)(param & 0xFFFFFFFFu);
                Mask keep = 0;
                RowPush<kR> acc;
                if (num == 0) {   // J >= 0: every pair of present values
                    keep = (vmask_j >> (24 + res)) & 1 ? rvalid(24 + res) : (Mask)0;
                } else if (P.gram[res].sig_words != 1) {
                    // four-word signature (long strings): the same bound, the
                    // intersection popcount summed over the words
                    const uint32_t restb = wb >> 16, rhs_b = opaque(__umul24(num, wb & 0xFFFFu));
                    uint32_t gjw[2 * kLongSigWords];
#pragma unroll
                    for (uint32_t w = 0; w < kLongSigWords; ++w) {
                        const uint64_t v = J64(gcol + w);
                        gjw[2 * w] = (uint32_t)v;
                        gjw[2 * w + 1] = (uint32_t)(v >> 32);
                    }
#pragma unroll
                    for (int r = kR - 1; r >= 0; --r) {
                        const uint64_t pr = pi0 + (uint64_t)r;
                        const uint32_t wa = f32[(jf32 + res) * n + pr];
                        uint32_t iub = min(wa >> 16, restb);
#pragma unroll
                        for (uint32_t w = 0; w < kLongSigWords; ++w) {
                            const uint64_t gi = f64[(gcol + w) * n + pr];
                            iub = popc_add((uint32_t)gi & gjw[2 * w], popc_add((uint32_t)(gi >> 32) & gjw[2 * w + 1], iub));
                        }
                        const bool ok = __umul24(iub, nd) >= num * (wa & 0xFFFFu) + rhs_b;
                        acc.push(r, __ballot(ok));
                    }
                    keep = acc.get();
                } else if (nd <= (1u << 18)) {
                    // num + den <= 2^18: I * (num + den) - num * |B| stays
                    // within int32, so one signed 24-bit multiply-add and a
                    // compare against the row's num * |A| (a scalar) decide
                    // the row
                    const uint32_t restb = wb >> 16;
                    const int neg_b = opaque(-(int)(num * (wb & 0xFFFFu)));
                    const uint32_t gj_lo = (uint32_t)gj, gj_hi = (uint32_t)(gj >> 32);
#pragma unroll
                    for (int r = kR - 1; r >= 0; --r) {
                        const uint64_t pr = pi0 + (uint64_t)r;
                        const uint32_t wa = f32[(jf32 + res) * n + pr];
                        const uint64_t gi = f64[gcol * n + pr];
                        const uint32_t rest = min(wa >> 16, restb);
                        const uint32_t iub = popc_add((uint32_t)gi & gj_lo, popc_add((uint32_t)(gi >> 32) & gj_hi, rest));
                        const int lhs = mad_i24((int)iub, (int)nd, neg_b);
                        acc.push(r, __ballot(lhs >= (int)(num * (wa & 0xFFFFu))));
                    }
                    keep = acc.get();
                } else {
                    const uint32_t restb = wb >> 16, rhs_b = opaque(__umul24(num, wb & 0xFFFFu));
                    const uint32_t gj_lo = (uint32_t)gj, gj_hi = (uint32_t)(gj >> 32);
#pragma unroll
                    for (int r = kR - 1; r >= 0; --r) {
                        const uint64_t pr = pi0 + (uint64_t)r;
                        const uint32_t wa = f32[(jf32 + res) * n + pr];
                        const uint64_t gi = f64[gcol * n + pr];
                        const uint32_t rest = min(wa >> 16, restb);
                        const uint32_t iub = popc_add((uint32_t)gi & gj_lo, popc_add((uint32_t)(gi >> 32) & gj_hi, rest));
                        const bool ok = __umul24(iub, nd) >= num * (wa & 0xFFFFu) + rhs_b;
                        acc.push(r, __ballot(ok));
                    }
                    keep = acc.get();
                }
                alive &= keep;
                work = 1;
                break;
            }
            default: {
                // exact similarity predicates, row by row, for rows where some
                // lane is still alive
                for (int r = 0; r < nr; ++r) {
                    const bool need = (alive >> r) & 1;
                    if (!__any(need)) continue;
                    const uint64_t pi = pi0 + r;
                    const uint32_t row_i = f32[pi];
                    const uint32_t vmask_i = f32[n + pi];
                    bool ok = false;
                    uint32_t w = 0;
                    if (op == OP_EQ_STR) {
                        const ColDev& c = P.cols[P.str_attr[res]];
                        const uint32_t li = f32[(str32 + res) * n + pi];
                        const uint32_t lj = J32(str32 + res);
                        if (need && li == lj) {
                            const uint8_t* si = c.bytes + c.off[row_i];
                            const uint8_t* sj = c.bytes + c.off[row_j];
                            ok = true;
                            w = li;
                            for (uint32_t x = 0; ok && x < li; ++x) ok = si[x] == sj[x];
                        }
                    } else if (op == OP_ED) {
                        const ColDev& c = P.cols[P.str_attr[res]];
                        const int m = (int)f32[(str32 + res) * n + pi];
                        const int nn = (int)J32(str32 + res);
                        const int k = (int)param;
                        const int words = m <= 32 ? 0 : (m + 63) / 64;
                        const bool run = need && abs(m - nn) <= k;
                        if (__any(run)) build_peq(peq, words, c.bytes + c.off[row_i], m, lane);
                        if (run) {
                            const uint8_t* tj = c.bytes + c.off[row_j];
                            int dist;
                            if constexpr (kLongEd) {
                                // patterns of up to four words, state in registers
                                dist = m == 0 ? nn : nn == 0 ? m
                                     : words == 0 ? myers<uint32_t, 1>((const uint32_t*)peq, m, tj, nn)
                                     : words == 1 ? myers<uint64_t, 1>((const uint64_t*)peq, m, tj, nn)
                                     : words == 2 ? myers<uint64_t, 2>((const uint64_t*)peq, m, tj, nn)
                                     : words == 3 ? myers<uint64_t, 3>((const uint64_t*)peq, m, tj, nn)
                                                  : myers<uint64_t, 4>((const uint64_t*)peq, m, tj, nn);
                            } else {
                                dist = myers_dispatch(peq, words, m, tj, nn, (uint64_t*)(wbase + P.lds_wave_myers),
                                                      lane);
                            }
                            ok = dist <= k;
                            w = (uint32_t)nn * (uint32_t)max(1, (m + 31) / 32);
                        }
                    } else {   // OP_JAC
                        const GramDev& g = P.gram[res];
                        const uint32_t ia = f32[(gram32 + res) * n + pi];
                        const uint32_t ca = ia & 0x7FFFFFFFu;
                        uint32_t* ig = (uint32_t*)(wbase + P.lds_wave_igram[res]);
                        if ((vmask_i >> (24 + res)) & 1) {
                            const uint32_t* src = g.codes + g.off[row_i];
                            for (uint32_t x = lane; x < ca; x += 64) ig[x] = src[x];
                            wave_sync();
                        }
                        if (need) {
                            const uint32_t jb = J32(gram32 + res);
                            const uint32_t cb = jb & 0x7FFFFFFFu;
                            const uint32_t I = intersect(ig, ca, (ia >> 31) != 0, g.codes + g.off[row_j], cb,
                                                         (jb >> 31) != 0);
                            const uint64_t U = (uint64_t)ca + cb - I;
                            ok = U == 0 || (uint64_t)I * (param & 0xFFFFFFFFu) >= (param >> 32) * U;
                            w = ca + cb;
                        }
                    }
                    if (need && !ok) alive &= ~((Mask)1 << r);
                    work += w;
                }
                break;
            }
            }
            if constexpr (kOrd) {   // a symmetric step narrows both valuations alike
                fwd &= alive;
                bwd &= alive;
            }
            if (guard) {   // the group's rules start from the pairs that passed
                base = alive;
                in_group = true;
                group_end = cp;
            }
            if constexpr (kCount) {
                // batches: this step ran once for the wave's 16-row batch
                uint32_t ev = 0, ps = 0;
                for (int r = 0; r < kR; ++r) {
                    ev += __popcll(__ballot((before >> r) & 1));
                    ps += __popcll(__ballot((alive >> r) & 1));
                }
                // filters: `waves` counts steps in the 16-row form, `work`
                // steps in the per-lane form
                const uint32_t waves = op <= OP_JACF && single ? 0u : 1u;
                uint32_t w = op <= OP_JACF ? 0u : work;
                for (int o = 32; o > 0; o >>= 1) w += __shfl_xor(w, o);
                if (op <= OP_JACF) w = single ? work : 0u;
                if (lane == 0) {
                    atomicAdd(&s_cnt[op * 4 + 0], (unsigned long long)waves);
                    atomicAdd(&s_cnt[op * 4 + 1], (unsigned long long)ev);
                    atomicAdd(&s_cnt[op * 4 + 2], (unsigned long long)ps);
                    atomicAdd(&s_cnt[op * 4 + 3], (unsigned long long)w);
                }
            }
            if (guard && !__any(alive != 0)) {   // no pair passed the shared step: past the group
                pc = cp;
                continue;
            }
            ++pc;
        }

        // ballot compaction of matched pairs, row by row (most batches
        // have none)
        if constexpr (kOrd) {
            // forward matches as (row, lane), backward ones as (lane, row)
            const int out_rows = __any((matched | matched_b) != 0) ? nr : 0;
            for (int r = 0; r < out_rows; ++r) {
                const uint64_t row_i = f32[pi0 + r];
#pragma unroll
                for (int dir = 0; dir < 2; ++dir) {
                    const bool m = (((dir == 0 ? matched : matched_b)) >> r) & 1;
                    const uint64_t mask = __ballot(m);
                    if (!mask) continue;
                    unsigned long long basev = 0;
                    if (lane == 0) basev = atomicAdd(P.counter, (unsigned long long)__popcll(mask));
                    basev = __shfl(basev, 0);
                    if (m) {
                        const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
                        const uint64_t pos = basev + __popcll(mask & lt);
                        if (pos < P.cap)
                            P.out[pos] = dir == 0 ? (row_i << 32) | row_j : ((uint64_t)row_j << 32) | row_i;
                    }
                }
            }
        }
        const int out_rows = kOrd ? 0 : __any(matched != 0) ? nr : 0;
        for (int r = 0; r < out_rows; ++r) {
            const bool m = (matched >> r) & 1;
            const uint64_t mask = __ballot(m);
            if (!mask) continue;
            const uint32_t row_i = f32[pi0 + r];
            unsigned long long basev = 0;
            if (lane == 0) basev = atomicAdd(P.counter, (unsigned long long)__popcll(mask));
            basev = __shfl(basev, 0);
            if (m) {
                const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
                const uint64_t pos = basev + __popcll(mask & lt);
                if (pos < P.cap) {
                    const uint64_t a = row_i < row_j ? row_i : row_j;
                    const uint64_t c = row_i < row_j ? row_j : row_i;
                    P.out[pos] = (a << 32) | c;
                }
            }
        }
    }
    if constexpr (kCount) {
        __syncthreads();
        for (uint32_t x = lane; x < kCountSlots; x += 64)
            if (s_cnt[x]) atomicAdd(&P.counts[x], s_cnt[x]);
    }
}

// Batch unit (tile * B + batch, B = 64 / rows batches per tile) of
// workgroup `bid` in a grid of a multiple of 32 workgroups.  Workgroups go
// round-robin to the 8 XCDs (bid % 8); XCD x runs tiles x, x + 8, x + 16,
// ... in order, the B batches of a tile back to back.  A tile's waves share
// its j-rows in one L2, and every XCD gets an even share of heavy and light
// tiles.
template <int kLogB = 2>
__device__ __forceinline__ uint64_t batch_unit(uint64_t bid) {
    const uint64_t x = bid & 7, g = bid >> 3;
    return (((g >> kLogB) * 8 + x) << kLogB) | (g & ((1u << kLogB) - 1u));
}

// One wave per workgroup, one batch of kR rows per wave (batch_unit), so no
// workgroup holds resources for waves that finished early.
template <bool kCount, int kR = kRows>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kR > 32 ? 7 : 8))) void k_match(
    const MatchParams P, const Instr* __restrict__ plan, const uint64_t* __restrict__ f64,
    const uint32_t* __restrict__ f32) {
    extern __shared__ __align__(16) uint8_t lds[];
    constexpr int kLogB = kR == 16 ? 2 : kR == 32 ? 1 : 0;
    const uint64_t w = batch_unit<kLogB>(blockIdx.x);
    const uint64_t t = w >> kLogB;
    if (t >= P.n_tiles) return;
    match_tile<kCount, false, false, kR>(P, gmem(plan), gmem(f64), gmem(f32), t, lds,
                                         (int)(w & ((1u << kLogB) - 1u)));
}

// k_match for partitions with edit-distance patterns past 64 bytes: the
// Myers state of up to four words lives in registers (no LDS for it, so
// more waves fit), at a register count the short-pattern kernel does not
// pay.
template <bool kCount, int kR = kRows>
__global__ __launch_bounds__(64) void k_match_long(const MatchParams P, const Instr* __restrict__ plan,
                                                   const uint64_t* __restrict__ f64,
                                                   const uint32_t* __restrict__ f32) {
    extern __shared__ __align__(16) uint8_t lds[];
    constexpr int kLogB = kR == 16 ? 2 : kR == 32 ? 1 : 0;
    const uint64_t w = batch_unit<kLogB>(blockIdx.x);
    const uint64_t t = w >> kLogB;
    if (t >= P.n_tiles) return;
    match_tile<kCount, true, false, kR>(P, gmem(plan), gmem(f64), gmem(f32), t, lds,
                                        (int)(w & ((1u << kLogB) - 1u)));
}

// k_match and k_match_long for ordered rule sets (no instrumented pass).
// At eight waves per SIMD the ordered kernel spills a few registers to
// scratch; a six-wave hint removes the spill but measured 5% slower.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(8))) void k_match_ord(
    const MatchParams P, const Instr* __restrict__ plan, const uint64_t* __restrict__ f64,
    const uint32_t* __restrict__ f32) {
    extern __shared__ __align__(16) uint8_t lds[];
    const uint64_t w = batch_unit(blockIdx.x);
    const uint64_t t = w >> 2;
    if (t >= P.n_tiles) return;
    match_tile<false, false, true>(P, gmem(plan), gmem(f64), gmem(f32), t, lds, (int)(w & 3));
}

__global__ __launch_bounds__(64) void k_match_long_ord(const MatchParams P, const Instr* __restrict__ plan,
                                                       const uint64_t* __restrict__ f64,
                                                       const uint32_t* __restrict__ f32) {
    extern __shared__ __align__(16) uint8_t lds[];
    const uint64_t w = batch_unit(blockIdx.x);
    const uint64_t t = w >> 2;
    if (t >= P.n_tiles) return;
    match_tile<false, true, true>(P, gmem(plan), gmem(f64), gmem(f32), t, lds, (int)(w & 3));
}

// partition of queue item x: prefix[p] <= x < prefix[p + 1]
__device__ inline uint32_t queue_partition(const uint64_t* __restrict__ prefix, uint32_t n_parts, uint64_t x) {
    uint32_t lo = 0, hi = n_parts;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (prefix[mid] <= x) lo = mid; else hi = mid;
    }
    return __builtin_amdgcn_readfirstlane(lo);
}

// Persistent grid over a queue of tiles of many partitions: each one-wave
// workgroup takes `grab` batch units (unit u = batch u % 4 of item u / 4)
// per atomic until the 4 x total units are gone.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(8))) void k_match_persistent(
    const MatchParams* __restrict__ mps, const uint64_t* __restrict__ prefix, uint32_t n_parts, uint64_t total,
    unsigned long long* cursor, uint32_t grab) {
    extern __shared__ __align__(16) uint8_t lds[];
    const uint64_t units = total * 4;
    for (;;) {
        unsigned long long got = 0;
        if (threadIdx.x == 0) got = atomicAdd(cursor, (unsigned long long)grab);
        got = __shfl(got, 0);
        // wave-uniform from here on: keep the queue walk on the scalar unit
        const uint64_t first = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(got >> 32)) << 32) |
                               __builtin_amdgcn_readfirstlane((uint32_t)got);
        if (first >= units) break;
        const uint64_t last = first + grab < units ? first + grab : units;
        for (uint64_t u = first; u < last; ++u) {
            const uint64_t item = u >> 2;
            const uint32_t p = queue_partition(prefix, n_parts, item);
            const MatchParams& P = mps[p];
            match_tile<false>(P, gmem(P.plan), gmem(P.feat.f64), gmem(P.feat.f32), item - prefix[p], lds,
                              (int)(u & 3));
        }
    }
}

// One one-wave workgroup per batch unit over the queue of many partitions
// (the hardware dispatcher hands out workgroups as compute units free up),
// mapped to XCDs as in k_match.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(8))) void k_match_multi(
    const MatchParams* __restrict__ mps, const uint64_t* __restrict__ prefix, uint32_t n_parts, uint64_t total) {
    extern __shared__ __align__(16) uint8_t lds[];
    const uint64_t u = batch_unit(blockIdx.x);
    const uint64_t item = u >> 2;
    if (item >= total) return;
    const uint32_t p = queue_partition(prefix, n_parts, item);
    const MatchParams& P = mps[p];
    match_tile<false>(P, gmem(P.plan), gmem(P.feat.f64), gmem(P.feat.f32), item - prefix[p], lds, (int)(u & 3));
}

// 16-byte stores over the aligned middle, byte stores at the ends.
__global__ void k_zero_bytes(uint8_t* p, size_t n) {
    const size_t lead = (16 - ((uintptr_t)p & 15)) & 15;
    const size_t head = lead < n ? lead : n;
    const size_t words = (n - head) / 16;
    const size_t tail = head + words * 16;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t x0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint4* w = (uint4*)(p + head);
    for (size_t x = x0; x < words; x += stride) w[x] = make_uint4(0u, 0u, 0u, 0u);
    if (x0 < head) p[x0] = 0;
    if (x0 < n - tail) p[tail + x0] = 0;
}

__global__ void k_fill_u64(unsigned long long* p, uint64_t n, unsigned long long v) {
    const uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x < n) p[x] = v;
}

// ------------------------------------------------------------ learned plan

// splitmix64 output function (Steele, Lea and Flood, OOPSLA 2014)
__device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ inline double wave_min(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}

// Exact filter of a predicate on two positions' features (the same bounds
// the plan's filter steps use).
__device__ inline bool feature_filter(const LearnParams& L, const PredSpec& sp, uint64_t pa, uint64_t pb) {
    const MatchParams& P = L.mp;
    const uint64_t n = P.feat.n;
    const uint64_t* f64 = P.feat.f64;
    const uint32_t* f32 = P.feat.f32;
    const uint32_t vb = f32[n + pa] & f32[n + pb];
    const uint32_t res = sp.res;
    switch (sp.op) {
    case OP_EQ_INT:
    case OP_ABSDIFF: {
        if (!((vb >> res) & 1)) return false;
        const int64_t a = (int64_t)f64[res * n + pa], b = (int64_t)f64[res * n + pb];
        return sp.op == OP_EQ_INT ? a == b : absdiff_le(a, b, (int64_t)sp.param);
    }
    case OP_EQ_STR:
    case OP_ED: {
        if (!((vb >> (16 + res)) & 1)) return false;
        const uint32_t la = f32[(2 + res) * n + pa], lb = f32[(2 + res) * n + pb];
        const uint64_t ca = f64[(P.n_int + res) * n + pa], cb = f64[(P.n_int + res) * n + pb];
        if (sp.op == OP_EQ_STR) return la == lb && ca == cb;
        const int k = (int)sp.param;
        return abs((int)la - (int)lb) <= k && max(__popcll(ca & ~cb), __popcll(cb & ~ca)) <= k;
    }
    default: {
        if (!((vb >> (24 + res)) & 1)) return false;
        const uint64_t sa = f32[(2 + P.n_str + res) * n + pa] & 0x7FFFFFFFu;
        const uint64_t sb = f32[(2 + P.n_str + res) * n + pb] & 0x7FFFFFFFu;
        const uint32_t gc = P.n_int + P.n_str + P.gram[res].sig_col;
        uint64_t ua = sa, ub = sb;
        for (uint32_t w = 0; w < P.gram[res].sig_words; ++w) {
            const uint64_t ga = f64[(gc + w) * n + pa], gb = f64[(gc + w) * n + pb];
            ua -= (uint64_t)__popcll(ga & ~gb);
            ub -= (uint64_t)__popcll(gb & ~ga);
        }
        const uint64_t iub = ua < ub ? ua : ub;
        const uint64_t num = sp.param >> 32, den = sp.param & 0xFFFFFFFFu;
        return iub * (num + den) >= num * (sa + sb);
    }
    }
}

// 16 features per (block, predicate): op one-hot (4), threshold relative to
// the data, threshold shape, log2 block size, length (or set size) mean / std /
// min / max, 3-bin length histogram, the fraction of adjacent position pairs
// passing the predicate's filter, mean signature density.  Statistics are
// taken over at most kFeatureSample evenly spaced positions of the block.
// One wave per listed block (workgroup g: block L.blocks[g], or block g
// without a list); the features go to row g.
__global__ __launch_bounds__(64) void k_block_features(const LearnParams L) {
    const MatchParams& P = L.mp;
    const uint32_t g = blockIdx.x;
    const uint32_t b = L.blocks ? L.blocks[g] : g;
    const uint32_t start = P.blk_start[b], nb = P.blk_size[b];
    const uint64_t n = P.feat.n;
    const uint64_t* f64 = P.feat.f64;
    const uint32_t* f32 = P.feat.f32;
    const uint32_t ns_pos = nb < kFeatureSample ? nb : kFeatureSample;
    for (uint32_t s = 0; s < L.n_spec; ++s) {
        const PredSpec sp = L.spec[s];
        const bool is_int = sp.op == OP_EQ_INT || sp.op == OP_ABSDIFF;
        const bool is_gram = sp.op == OP_JAC;
        double cnt = 0, sum = 0, sum2 = 0, mn = 1e300, mx = -1e300, b0 = 0, b1 = 0, b2 = 0, pops = 0, pass = 0;
        // statistics over at most kFeatureSample evenly spaced positions
        for (uint32_t u = threadIdx.x; u < ns_pos; u += 64) {
            const uint32_t x = (uint32_t)(((uint64_t)u * nb) / ns_pos);
            const uint64_t pos = (uint64_t)start + x;
            const uint32_t vm = f32[n + pos];
            double lv = 0.0;
            bool v;
            if (is_int) {
                v = (vm >> sp.res) & 1;
                lv = (double)(int64_t)f64[sp.res * n + pos];
            } else if (!is_gram) {
                v = (vm >> (16 + sp.res)) & 1;
                lv = (double)f32[(2 + sp.res) * n + pos];
                if (v) pops += __popcll(f64[(P.n_int + sp.res) * n + pos]);
            } else {
                v = (vm >> (24 + sp.res)) & 1;
                lv = (double)(f32[(2 + P.n_str + sp.res) * n + pos] & 0x7FFFFFFFu);
                if (v) pops += __popcll(f64[(P.n_int + P.n_str + P.gram[sp.res].sig_col) * n + pos]);
            }
            if (v) {
                cnt += 1;
                sum += lv;
                sum2 += lv * lv;
                mn = fmin(mn, lv);
                mx = fmax(mx, lv);
                if (!is_int) {
                    if (lv < 16) b0 += 1; else if (lv < 48) b1 += 1; else b2 += 1;
                }
            }
            if (x + 1 < nb && feature_filter(L, sp, pos, pos + 1)) pass += 1;
        }
        cnt = wave_sum(cnt);
        sum = wave_sum(sum);
        sum2 = wave_sum(sum2);
        mn = wave_min(mn);
        mx = -wave_min(-mx);
        b0 = wave_sum(b0);
        b1 = wave_sum(b1);
        b2 = wave_sum(b2);
        pops = wave_sum(pops);
        pass = wave_sum(pass);
        if (threadIdx.x == 0) {
            float* f = L.features + ((size_t)g * L.n_spec + s) * kFeatures;
            const double c = cnt > 0 ? cnt : 1.0;
            const double mean = sum / c;
            const double sd = sqrt(fmax(sum2 / c - mean * mean, 0.0));
            const int hop = sp.op == OP_EQ_INT || sp.op == OP_EQ_STR ? 0 : sp.op == OP_ED ? 1 : sp.op == OP_JAC ? 2 : 3;
            for (int k = 0; k < 4; ++k) f[k] = k == hop ? 1.f : 0.f;
            double thr = 0, shape = 0;
            if (sp.op == OP_ED) {
                thr = (double)sp.param / fmax(1.0, mean);
                shape = fmin((double)sp.param, 64.0) / 16.0;
            } else if (sp.op == OP_JAC) {
                thr = (double)(sp.param >> 32) / (double)(sp.param & 0xFFFFFFFFu);
                shape = 0.25 * (double)P.gram[sp.res].q;
            } else if (sp.op == OP_ABSDIFF) {
                thr = (double)sp.param / (1.0 + sd);
                shape = log2(1.0 + (double)sp.param) / 64.0;
            }
            f[4] = (float)fmin(thr, 16.0);
            f[5] = (float)shape;
            f[6] = (float)(log2((double)nb) / 16.0);
            if (is_int) {
                f[7] = (float)(log2(1.0 + fabs(mean)) / 64.0);
                f[8] = (float)(log2(1.0 + sd) / 64.0);
                f[9] = f[10] = f[11] = f[12] = f[13] = 0.f;
            } else {
                f[7] = (float)(mean / 64.0);
                f[8] = (float)(sd / 64.0);
                f[9] = (float)((cnt > 0 ? mn : 0.0) / 64.0);
                f[10] = (float)((cnt > 0 ? mx : 0.0) / 64.0);
                f[11] = (float)(b0 / c);
                f[12] = (float)(b1 / c);
                f[13] = (float)(b2 / c);
            }
            f[14] = (float)(pass / (double)(ns_pos - (ns_pos == nb ? 1 : 0)));
            f[15] = (float)(pops / c / 64.0);
        }
    }
}

// Logging pass: wave (b, s) evaluates every predicate, in isolation and
// without short-circuit, on 64 sampled pairs of block b:
//   c = seed + ((b * samples + s) << 7),
//   i = mix64(c + 64) mod n_b, j_l = mix64(c + l) mod n_b (l = lane; j_l = i
//   is replaced by (i + 1) mod n_b), positions inside the block.
// It accumulates per (block, predicate) the lanes, the lanes that satisfy
// the predicate, the wave's clock cycles spent on the exact check of every
// lane whose values are present (not gated by the filter) and the lanes
// that pass the predicate's first plan step (its exact filter; for value
// predicates the predicate itself).
__global__ __launch_bounds__(64) void k_log_samples(const LearnParams L) {
    extern __shared__ __align__(16) uint8_t lds[];
    const MatchParams& P = L.mp;
    const int lane = threadIdx.x;
    const uint32_t b = blockIdx.x, s = blockIdx.y;
    const uint32_t start = P.blk_start[b], nb = P.blk_size[b];
    const uint64_t n = P.feat.n;
    const uint32_t* f32 = P.feat.f32;
    const uint64_t c = L.seed + (((uint64_t)b * L.samples + s) << 7);
    const uint32_t ip = (uint32_t)(mix64(c + 64) % nb);
    uint32_t jp = (uint32_t)(mix64(c + (uint64_t)lane) % nb);
    if (jp == ip) jp = (jp + 1) % nb;
    const uint64_t pi = (uint64_t)start + ip, pj = (uint64_t)start + jp;
    const uint32_t row_i = f32[pi], row_j = f32[pj];
    const uint32_t vmask_i = f32[n + pi];
    const uint32_t vb = vmask_i & f32[n + pj];
    uint8_t* peq = lds + P.lds_wave_peq;
    for (uint32_t x = 0; x < L.n_spec; ++x) {
        const PredSpec sp = L.spec[x];
        const uint32_t res = sp.res;
        const bool first = feature_filter(L, sp, pi, pj);
        const uint64_t filtered = __popcll(__ballot(first));
        const uint64_t t0 = __builtin_readcyclecounter();
        bool r = false;
        if (sp.op == OP_EQ_INT || sp.op == OP_ABSDIFF) {
            r = feature_filter(L, sp, pi, pj);
        } else if (sp.op == OP_EQ_STR) {
            const ColDev& col = P.cols[P.str_attr[res]];
            const uint32_t li = f32[(2 + res) * n + pi], lj = f32[(2 + res) * n + pj];
            if (((vb >> (16 + res)) & 1) && li == lj) {
                const uint8_t* si = col.bytes + col.off[row_i];
                const uint8_t* sj = col.bytes + col.off[row_j];
                r = true;
                for (uint32_t q = 0; r && q < li; ++q) r = si[q] == sj[q];
            }
        } else if (sp.op == OP_ED) {
            const ColDev& col = P.cols[P.str_attr[res]];
            const bool valid = (vb >> (16 + res)) & 1;
            const int m = (int)f32[(2 + res) * n + pi];
            const int nn = (int)f32[(2 + res) * n + pj];
            const int words = m <= 32 ? 0 : (m + 63) / 64;
            if (__any(valid)) build_peq(peq, words, col.bytes + col.off[row_i], m, lane);
            if (valid) {
                const int dist = myers_dispatch(peq, words, m, col.bytes + col.off[row_j], nn,
                                                (uint64_t*)(lds + P.lds_wave_myers), lane);
                r = dist <= (int)sp.param;
            }
        } else {   // OP_JAC
            const GramDev& g = P.gram[res];
            const bool valid = (vb >> (24 + res)) & 1;
            const uint32_t ia = f32[(2 + P.n_str + res) * n + pi];
            const uint32_t ca = ia & 0x7FFFFFFFu;
            uint32_t* ig = (uint32_t*)(lds + P.lds_wave_igram[res]);
            if ((vmask_i >> (24 + res)) & 1) {
                const uint32_t* src = g.codes + g.off[row_i];
                for (uint32_t q = lane; q < ca; q += 64) ig[q] = src[q];
                wave_sync();
            }
            if (valid) {
                const uint32_t jb = f32[(2 + P.n_str + res) * n + pj];
                const uint32_t cb = jb & 0x7FFFFFFFu;
                const uint32_t I = intersect(ig, ca, (ia >> 31) != 0, g.codes + g.off[row_j], cb, (jb >> 31) != 0);
                const uint64_t U = (uint64_t)ca + cb - I;
                r = U == 0 || (uint64_t)I * (sp.param & 0xFFFFFFFFu) >= (sp.param >> 32) * U;
            }
        }
        const uint64_t passed = __popcll(__ballot(r));
        const uint64_t t1 = __builtin_readcyclecounter();
        if (lane == 0) {
            unsigned long long* cnt = L.counts + ((size_t)b * L.n_spec + x) * 4;
            atomicAdd(&cnt[0], 64ull);
            atomicAdd(&cnt[1], (unsigned long long)passed);
            atomicAdd(&cnt[2], (unsigned long long)(t1 - t0));
            atomicAdd(&cnt[3], (unsigned long long)filtered);
        }
    }
}

// ------------------------------------------------------------ per-pair cost network

__device__ inline bool col_valid(const ColDev& c, uint32_t r) {
    return c.valid == nullptr || ((c.valid[r >> 3] >> (r & 7)) & 1);
}

// Sampled pair s of D x D (n >= 2 rows).
__device__ inline void sample_pair(uint64_t seed, uint32_t s, uint32_t n, uint32_t& i, uint32_t& j) {
    i = (uint32_t)(mix64(seed + 2ull * s) % n);
    j = (uint32_t)(mix64(seed + 2ull * s + 1) % n);
    if (j == i) j = (i + 1) % n;
}

// The per-pair network's 16 inputs for predicate sp on rows (i, j):
// one-hot kind (0-4), presence of both values (5, 6), byte lengths / 64
// (7, 8), a kind-specific pair (9, 10: equal lengths for string equality;
// pattern words / 4 and k / 16 for edit distance; q-gram counts / 64 for
// Jaccard), Jaccard's short-string flag (11) and threshold (12), the
// shorter length and the length difference / 64 (13, 14), and 1 (15).
// Every value is an integer times a power of two, or one rounded fraction.
__device__ inline void pair_features(const PairParams& P, const PairSpec& sp, uint32_t i, uint32_t j, float* f) {
#pragma unroll
    for (int k = 5; k < kFeatures; ++k) f[k] = 0.f;
    const ColDev& c = P.cols[sp.attr];
    const bool ok1 = col_valid(c, i), ok2 = col_valid(c, j);
#pragma unroll
    for (int k = 0; k < 5; ++k) f[k] = sp.kind == k ? 1.f : 0.f;
    f[5] = ok1 ? 1.f : 0.f;
    f[6] = ok2 ? 1.f : 0.f;
    f[15] = 1.f;
    if (sp.kind == PK_VALUE_EQ || sp.kind == PK_ABSDIFF) return;
    const uint32_t l1 = ok1 ? (uint32_t)(c.off[i + 1] - c.off[i]) : 0u;
    const uint32_t l2 = ok2 ? (uint32_t)(c.off[j + 1] - c.off[j]) : 0u;
    const float s64 = 1.f / 64.f;
    f[7] = (float)l1 * s64;
    f[8] = (float)l2 * s64;
    f[13] = (float)min(l1, l2) * s64;
    f[14] = (float)(l1 > l2 ? l1 - l2 : l2 - l1) * s64;
    if (sp.kind == PK_STRING_EQ) {
        f[9] = (ok1 && ok2 && l1 == l2) ? 1.f : 0.f;
    } else if (sp.kind == PK_EDIT) {
        f[9] = (float)(l1 <= 32 ? 0u : (l1 + 63) / 64) * 0.25f;
        f[10] = (float)sp.k * (1.f / 16.f);
    } else {
        const GramDev& g = P.gram[sp.gram];
        f[9] = (float)(ok1 ? g.cnt[i] : 0u) * s64;
        f[10] = (float)(ok2 ? g.cnt[j] : 0u) * s64;
        f[11] = ((l1 > 0 && l1 < sp.q) || (l2 > 0 && l2 < sp.q)) ? 1.f : 0.f;
        f[12] = (float)((double)sp.num / (double)sp.den);
    }
}

// The exact check of predicate sp on rows (i, j), every lane on that pair
// (ok: both values present, uniform across the wave).
__device__ inline bool check_pair(const PairParams& P, const PairSpec& sp, uint32_t i, uint32_t j, bool ok,
                                  uint8_t* lds, int lane) {
    if (!ok) return false;
    const ColDev& c = P.cols[sp.attr];
    if (sp.kind == PK_VALUE_EQ) return c.values[i] == c.values[j];
    if (sp.kind == PK_ABSDIFF) return absdiff_le(c.values[i], c.values[j], sp.d);
    if (sp.kind == PK_STRING_EQ) {
        const uint32_t l1 = (uint32_t)(c.off[i + 1] - c.off[i]), l2 = (uint32_t)(c.off[j + 1] - c.off[j]);
        if (l1 != l2) return false;
        const uint8_t* a = c.bytes + c.off[i];
        const uint8_t* b = c.bytes + c.off[j];
        bool r = true;
        for (uint32_t q = 0; r && q < l1; ++q) r = a[q] == b[q];
        return r;
    }
    if (sp.kind == PK_EDIT) {
        const int m = (int)(c.off[i + 1] - c.off[i]), nn = (int)(c.off[j + 1] - c.off[j]);
        const int words = m <= 32 ? 0 : (m + 63) / 64;   // <= kMaxEdWords: compile bounds the length
        build_peq(lds + kPairLdsPeq, words, c.bytes + c.off[i], m, lane);
        const int dist = myers_dispatch(lds + kPairLdsPeq, words, m, c.bytes + c.off[j], nn,
                                        (uint64_t*)(lds + kPairLdsMyers), lane);
        return dist <= (int)sp.k;
    }
    const GramDev& g = P.gram[sp.gram];
    const uint32_t ca = g.cnt[i], cb = g.cnt[j];   // ca <= max_cnt: the LDS holds it
    uint32_t* ig = (uint32_t*)(lds + kPairLdsGrams);
    const uint32_t* src = g.codes + g.off[i];
    for (uint32_t q = lane; q < ca; q += 64) ig[q] = src[q];
    wave_sync();
    const uint32_t I = intersect(ig, ca, (g.flags[i] & 1) != 0, g.codes + g.off[j], cb, (g.flags[j] & 1) != 0);
    wave_sync();   // the list is rewritten by a following check
    const uint64_t U = (uint64_t)ca + cb - I;
    return U == 0 || (uint64_t)I * sp.den >= (uint64_t)sp.num * U;
}

// Logging pass of the per-pair network: workgroup (s, x), one wave,
// checks predicate x on sampled pair s with every lane on that same pair,
// so the wave's clock cycles around the check are the time of checking one
// pair (edit distance: the pattern table and Myers' scan; Jaccard: staging
// row i's q-gram list and the merge).  The check runs twice: the first
// brings the pair's values into the caches, as the match kernel's staged
// reads do; the second is timed, less the cycles of an empty interval
// between two clock reads (the clock's own cost), floored at 0.
__global__ __launch_bounds__(64) void k_pair_log(const PairParams P) {
    extern __shared__ __align__(16) uint8_t lds[];
    const int lane = threadIdx.x;
    const uint32_t s = blockIdx.x, x = blockIdx.y;
    const PairSpec sp = P.spec[x];
    uint32_t i, j;
    sample_pair(P.seed, s, P.n_rows, i, j);
    const size_t row = (size_t)x * P.samples + s;
    if (lane == 0) {
        float f[kFeatures];
        pair_features(P, sp, i, j, f);
        float4* dst = (float4*)(P.features + row * kFeatures);
#pragma unroll
        for (int k = 0; k < 4; ++k) dst[k] = make_float4(f[4 * k], f[4 * k + 1], f[4 * k + 2], f[4 * k + 3]);
        if (P.pairs && x == 0) {
            P.pairs[2 * (size_t)s] = i;
            P.pairs[2 * (size_t)s + 1] = j;
        }
    }
    const ColDev& c = P.cols[sp.attr];
    const bool ok = col_valid(c, i) && col_valid(c, j);   // uniform: one pair per wave
    const uint64_t warm = __ballot(check_pair(P, sp, i, j, ok, lds, lane));
    const uint64_t e0 = __builtin_readcyclecounter();
    const uint64_t e1 = __builtin_readcyclecounter();
    const uint64_t t0 = __builtin_readcyclecounter();
    const bool r = check_pair(P, sp, i, j, ok, lds, lane);
    const uint64_t passed = __ballot(r);
    const uint64_t t1 = __builtin_readcyclecounter();
    if (lane == 0) {
        const uint64_t spent = t1 - t0, clock = e1 - e0;
        P.sat[row] = (passed && warm) ? 1u : 0u;
        P.cycles[row] = (unsigned long long)(spent > clock ? spent - clock : 0);
    }
}

// Features of every (predicate, sampled pair) row, one thread per row.
__global__ __launch_bounds__(256) void k_pair_features(const PairParams P) {
    const uint64_t t = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (uint64_t)P.n_spec * P.samples) return;
    const uint32_t x = (uint32_t)(t / P.samples), s = (uint32_t)(t % P.samples);
    uint32_t i, j;
    sample_pair(P.seed, s, P.n_rows, i, j);
    float f[kFeatures];
    pair_features(P, P.spec[x], i, j, f);
    float4* dst = (float4*)(P.features + t * kFeatures);
#pragma unroll
    for (int k = 0; k < 4; ++k) dst[k] = make_float4(f[4 * k], f[4 * k + 1], f[4 * k + 2], f[4 * k + 3]);
}

// Summed estimate of predicate x (workgroup x): the network's second
// output y is log2(1 + cycles) / 16, so a row estimates
// 2^(16 * clamp(y, 0, 4)) - 1 cycles (NaN counts as 0).  Fixed-order fp64
// sums, so equal inputs give equal costs.
__global__ __launch_bounds__(256) void k_pair_sum(const PairParams P) {
    __shared__ double part[256];
    const uint32_t x = blockIdx.x;
    double acc = 0.0;
    for (uint32_t s = threadIdx.x; s < P.samples; s += 256) {
        const double y = (double)P.y[((size_t)x * P.samples + s) * 2 + 1];
        const double t = fmin(fmax(y, 0.0), 4.0);
        acc += exp2(16.0 * t) - 1.0;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) P.sums[x] = part[0];
}

// ------------------------------------------------------------ plan choice

// The shape of a block's wave batches: rows per batch, lanes, and the
// per-lane form's threshold (a filter step runs lane by lane, one live row
// per round, when no lane has more live rows than that).
struct BatchShape {
    float rows, lanes;
    int sparse;
};

__device__ inline BatchShape batch_shape(uint32_t nb, uint32_t rows, uint32_t sparse_setting) {
    BatchShape b;
    b.rows = (float)min(nb, rows);
    b.lanes = (float)min(nb, (uint32_t)kTile);
    b.sparse = (int)min(min(sparse_rows(sparse_setting, rows), (uint32_t)kMaxSparseRows), min(nb, rows) >> 1);
    return b;
}

// First-stage step cost per row, in the library's lane-op units.
__device__ inline float first_cost(uint8_t op) {
    switch (op) {
    case OP_EQ_INT: return 1.f;
    case OP_ABSDIFF: return 4.f;
    case OP_EQ_STR: return 3.f;
    default: return 12.f;
    }
}

// Cost of one round of the per-lane form against one row of the batch form
// (per-lane loads instead of scalar ones, and the round's control).
constexpr float kSparseRound = 2.f;
// Fixed cost of running a step at all (instruction fetch and decode, the
// wave-wide tests, the lane's feature loads), in the same units: measured
// at about 20 rows of a signature filter's 12, so a step the batch never
// reaches saves far more than a cheaper step it does.
constexpr float kStepFixed = 240.f;

// Expected cost of a first-stage step of per-row cost c reached with
// per-pair survival probability s (each pair independently): the fixed cost
// when some pair of the batch is alive (probability 1 - (1 - s)^pairs),
// plus, with X the live rows of a lane, X ~ Binomial(rows, s), the batch
// form's c x rows when some lane has more than `sparse` live rows; otherwise
// the per-lane form takes one round per live row of the fullest lane, so the
// variable part is c (rows (1 - A_T) + kSparseRound sum_{m < T} (A_T - A_m))
// with A_m = P(X <= m)^lanes.  The plan choice only ranks alternatives, so
// single precision and fast intrinsics do.
__device__ inline float step_cost(float c, float s, const BatchShape& b) {
    if (s <= 0.f) return 0.f;
    const float any = s >= 1.f ? 1.f : 1.f - __expf(b.rows * b.lanes * __logf(1.f - s));
    const int T = b.sparse;
    // F_m = P(X <= m) and A_m = F_m^lanes, accumulated in one pass (no
    // array): sum_{m<T} (A_T - A_m) = T A_T - sum_{m<T} A_m
    auto A = [&](float F) { return F <= 0.f ? 0.f : F >= 1.f ? 1.f : __expf(b.lanes * __logf(F)); };
    float sum_a = 0.f, at;
    if (s >= 1.f) {
        for (int m = 0; m < T; ++m) sum_a += (float)m >= b.rows ? 1.f : 0.f;
        at = (float)T >= b.rows ? 1.f : 0.f;
    } else {
        const float q = 1.f - s;
        float pm = __expf(b.rows * __logf(q));   // P(X = 0)
        float F = pm;
        for (int m = 1; m <= T; ++m) {
            sum_a += A(F);   // A_{m-1}
            pm = (float)m <= b.rows ? pm * (b.rows - (float)(m - 1)) / (float)m * (s / q) : 0.f;
            F = fminf(1.f, F + pm);
        }
        at = A(F);
    }
    const float rounds = (float)T * at - sum_a;
    return kStepFixed * any + c * (b.rows * (1.f - at) + kSparseRound * rounds);
}

struct BlockEst {
    const float* y;
    __device__ float pass(uint32_t s) const {
        const float v = y[2 * s];
        return isfinite(v) ? fminf(1.f, fmaxf(0.f, v)) : 1.f;
    }
};

// Expected first-stage cost of a wave batch running a rule's steps in
// order `ord` (indices into the rule's steps).
__device__ inline float stage_cost(const PlanChoiceParams& C, uint32_t r, const uint8_t* ord, int len,
                                   const BlockEst& e, const BatchShape& b) {
    // a rule under a shared guard step starts from the pairs that passed it
    float total = 0.f, surv = C.rule_guard[r] == 0xFF ? 1.f : e.pass(C.rule_guard[r]);
    for (int k = 0; k < len; ++k) {
        const uint32_t sx = C.rule_spec[r][ord[k]];
        total += step_cost(first_cost(C.spec_kind[sx]), surv, b);
        surv *= e.pass(sx);
    }
    return total;
}

__device__ inline uint64_t pack_order(const uint8_t* ord, int len) {
    uint64_t code = 0;
    for (int k = 0; k < len; ++k) code |= (uint64_t)(ord[k] + 1) << (4 * k);
    return code;
}

// Per block and rule: the first-stage order.  Steps after the first run
// mostly in the per-lane form, whose cost follows the pairs still alive, so
// they are ranked by cost / (1 - pass rate) ascending (the order that
// minimises the expected cost of independent filters paid per pair); every
// step is tried as the first one (the batch form's cost), and the cheapest
// order under stage_cost is taken when the model expects it at least 10%
// cheaper than the heuristic order.
__device__ inline void rule_choice(const PlanChoiceParams& C, uint32_t r, const BlockEst& e, const BatchShape& b,
                                   uint8_t* fo, float* cost_heuristic = nullptr, float* cost_chosen = nullptr) {
    const int len = C.rule_len[r];
    uint8_t id[kMaxRuleSteps], lo[kMaxRuleSteps], cand[kMaxRuleSteps];
    float rank[kMaxRuleSteps];
    for (int k = 0; k < len; ++k) {
        id[k] = (uint8_t)k;
        lo[k] = (uint8_t)k;
        const uint32_t sx = C.rule_spec[r][k];
        rank[k] = first_cost(C.spec_kind[sx]) / fmaxf(1e-20f, 1.f - e.pass(sx));
    }
    for (int a = 1; a < len; ++a)   // stable insertion sort by rank
        for (int k = a; k > 0 && rank[lo[k]] < rank[lo[k - 1]]; --k) {
            const uint8_t t = lo[k]; lo[k] = lo[k - 1]; lo[k - 1] = t;
        }
    float best = 3.0e38f;
    uint8_t best_first = lo[0];
    for (int f = 0; f < len; ++f) {   // candidate first step lo[f], the rest in rank order
        cand[0] = lo[f];
        for (int k = 0, o = 1; k < len; ++k)
            if (k != f) cand[o++] = lo[k];
        const float cost = stage_cost(C, r, cand, len, e, b);
        if (cost < best) {
            best = cost;
            best_first = lo[f];
        }
    }
    cand[0] = best_first;
    for (int k = 0, o = 1; k < len; ++k)
        if (lo[k] != best_first) cand[o++] = lo[k];
    const float heur = stage_cost(C, r, id, len, e, b);
    const bool take = best < 0.9f * heur;
    for (int k = 0; k < len; ++k) fo[k] = take ? cand[k] : id[k];
    if (cost_heuristic) *cost_heuristic += heur;
    if (cost_chosen) *cost_chosen += take ? best : heur;
    // the exact checks keep the heuristic's order, whatever the first-stage
    // order: the model predicts their cost but not how many pairs they
    // reject, and a cost-only order can put a check that passes nearly
    // every pair ahead of a selective one
}

// The first block to claim a slot writes its plan: the heuristic plan with
// each rule's first-stage steps (at the start of its segment) in the chosen
// order; exact checks, checkpoints and guard steps keep their places.
__device__ inline void write_plan(const PlanChoiceParams& C, uint32_t x, const BlockEst& e, const BatchShape& batch) {
    Instr* dst = C.code + (size_t)x * C.plan_len;
    const Instr* base = C.code;
    for (uint32_t i = 0; i < C.plan_len; ++i) dst[i] = base[i];
    for (uint32_t r = 0; r < C.n_rules; ++r) {
        uint8_t fo[kMaxRuleSteps];
        rule_choice(C, r, e, batch, fo);
        const uint32_t seg = C.rule_seg[r];
        for (int k = 0; k < (int)C.rule_len[r]; ++k) dst[seg + k] = base[seg + fo[k]];
    }
}

// One thread per block: for every rule, the first-stage order of
// rule_choice (exact checks keep the heuristic's order).  Writes the
// block's plan slot.
__global__ __launch_bounds__(64) void k_plan_choice(const PlanChoiceParams C) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    bool learned = false, overflow = false, wrote = false;
    float cost_h = 0.f, cost_c = 0.f;   // this block's predicted cost under either plan
    if (g < C.n_blocks) {
        const uint32_t b = C.blocks[g];
        const BatchShape batch = batch_shape(C.blk_size[b], C.rows, C.sparse_rows);
        BlockEst e{C.y + (size_t)g * C.n_spec * 2};
        uint64_t h = 0x6A09E667F3BCC909ull;
        float heur = 0.f, chosen = 0.f;   // predicted cost per wave batch, both plans
        {
            for (uint32_t r = 0; r < C.n_rules; ++r) {
                uint8_t fo[kMaxRuleSteps];
                rule_choice(C, r, e, batch, fo, &heur, &chosen);
                const int len = C.rule_len[r];
                bool same = true;
                for (int k = 0; k < len; ++k) same &= fo[k] == k;
                if (!same) {
                    learned = true;
                    h = mix64(h ^ ((uint64_t)(r + 1) << 56) ^ pack_order(fo, len));
                }
            }
        }
        // the block's predicted cost under either plan, weighted by its
        // wave batches (its pairs over the pairs of a batch)
        const float nbf = (float)C.blk_size[b];
        const float w = 0.5f * nbf * (nbf - 1.f) / (batch.rows * batch.lanes);
        cost_h = w * heur;
        cost_c = w * chosen;
        uint32_t slot = 0;
        if (learned) {
            const unsigned long long key = h ? h : 1ull;
            const uint32_t mask = C.n_slots - 1;
            uint32_t x = (uint32_t)(key & mask);
            for (uint32_t probe = 0; probe < C.n_slots; ++probe, x = (x + 1) & mask) {
                if (x == 0) continue;   // slot 0 is the heuristic plan
                // most blocks find their choice already present: read first,
                // and only try to claim an empty slot
                unsigned long long cur = __hip_atomic_load(&C.keys[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (cur == 0ull) {
                    cur = atomicCAS(&C.keys[x], 0ull, key);
                    if (cur == 0ull) {
                        write_plan(C, x, e, batch);
                        wrote = true;
                        slot = x;
                        break;
                    }
                }
                if (cur == key) {
                    slot = x;
                    break;
                }
            }
            overflow = slot == 0;
            learned = slot != 0;
        }
        C.blk_slot[b] = slot;
    }
    // one atomic per wave for the partition's totals
    for (int o = 32; o > 0; o >>= 1) {
        cost_h += __shfl_xor(cost_h, o);
        cost_c += __shfl_xor(cost_c, o);
    }
    if ((threadIdx.x & 63) == 0 && (cost_h != 0.f || cost_c != 0.f)) {
        atomicAdd(&C.cost[0], cost_h);
        atomicAdd(&C.cost[1], cost_c);
    }
    const uint64_t nl = __popcll(__ballot(learned)), no = __popcll(__ballot(overflow));
    const uint64_t nw = __popcll(__ballot(wrote));
    if ((threadIdx.x & 63) == 0) {
        if (nl) atomicAdd(&C.stats[0], (unsigned long long)nl);
        if (no) atomicAdd(&C.stats[1], (unsigned long long)no);
        if (nw) atomicAdd(&C.stats[2], (unsigned long long)nw);
    }
}

}  // namespace

// Raises a kernel's dynamic-LDS limit once it needs more than 64 KB.
static hipError_t allow_lds(const void* fn, int* configured, uint32_t bytes) {
    if (bytes <= 65536 || *configured >= (int)bytes) return hipSuccess;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess) *configured = (int)bytes;
    return e;
}

// The plain kernels at kR rows per batch (64 / kR batches per tile).
template <int kR>
static hipError_t launch_match_rows(const MatchParams& p, hipStream_t s) {
    static int configured[4] = {0, 0, 0, 0};
    const unsigned grid = (unsigned)((p.n_tiles * (kTile / kR) + 31) & ~31ull);   // batch_unit: multiple of 32
    if (p.ed_words >= 2) {   // the register-state kernel leaves out the LDS Myers region
        MatchParams q = p;
        q.lds_counts = p.lds_wave_myers;
        q.lds_bytes = (q.lds_counts + (p.counts ? kCountSlots * 8 : 0) + 15) & ~15u;
        const void* fn = p.counts ? (const void*)k_match_long<true, kR> : (const void*)k_match_long<false, kR>;
        hipError_t e = allow_lds(fn, &configured[p.counts ? 2 : 1], q.lds_bytes);
        if (e != hipSuccess) return e;
        if (p.counts)
            k_match_long<true, kR><<<grid, 64, q.lds_bytes, s>>>(q, q.plan, q.feat.f64, q.feat.f32);
        else
            k_match_long<false, kR><<<grid, 64, q.lds_bytes, s>>>(q, q.plan, q.feat.f64, q.feat.f32);
        return hipGetLastError();
    }
    const void* fn = p.counts ? (const void*)k_match<true, kR> : (const void*)k_match<false, kR>;
    hipError_t e = allow_lds(fn, &configured[p.counts ? 3 : 0], p.lds_bytes);
    if (e != hipSuccess) return e;
    if (p.counts)
        k_match<true, kR><<<grid, 64, p.lds_bytes, s>>>(p, p.plan, p.feat.f64, p.feat.f32);
    else
        k_match<false, kR><<<grid, 64, p.lds_bytes, s>>>(p, p.plan, p.feat.f64, p.feat.f32);
    return hipGetLastError();
}

hipError_t launch_match(const MatchParams& p, hipStream_t s) {
    if (p.n_tiles == 0) return hipSuccess;
    if (p.n_tiles > kMaxTiles) return hipErrorInvalidValue;   // the grid holds 4 x n_tiles workgroups
    static int configured[6] = {0, 0, 0, 0, 0, 0};
    const unsigned grid = (unsigned)((p.n_tiles * 4 + 31) & ~31ull);   // batch_unit needs a multiple of 32
    if (p.ordered) {
        if (p.counts) return hipErrorInvalidValue;   // no instrumented pass for ordered rule sets
        if (p.ed_words >= 2) {
            MatchParams q = p;
            q.lds_counts = p.lds_wave_myers;
            q.lds_bytes = (q.lds_counts + 15) & ~15u;
            hipError_t e = allow_lds((const void*)k_match_long_ord, &configured[5], q.lds_bytes);
            if (e != hipSuccess) return e;
            k_match_long_ord<<<grid, 64, q.lds_bytes, s>>>(q, q.plan, q.feat.f64, q.feat.f32);
        } else {
            hipError_t e = allow_lds((const void*)k_match_ord, &configured[4], p.lds_bytes);
            if (e != hipSuccess) return e;
            k_match_ord<<<grid, 64, p.lds_bytes, s>>>(p, p.plan, p.feat.f64, p.feat.f32);
        }
        return hipGetLastError();
    }
    // 32- or 64-row batches (two or one per tile) for the plain kernels and
    // their instrumented pass when asked: a step's fixed cost is paid once
    // per 2,048 or 4,096 pairs instead of 1,024
    if (p.rows == 64) return launch_match_rows<64>(p, s);
    const bool r32 = p.rows == 32;
    const unsigned grid32 = (unsigned)((p.n_tiles * 2 + 31) & ~31ull);
    static int configured32[4] = {0, 0, 0, 0};
    if (p.ed_words >= 2) {
        // the register-state kernel leaves out the LDS Myers region (the
        // layout's last one)
        MatchParams q = p;
        q.lds_counts = p.lds_wave_myers;
        q.lds_bytes = (q.lds_counts + (p.counts ? kCountSlots * 8 : 0) + 15) & ~15u;
        if (r32) {
            const void* fn = p.counts ? (const void*)k_match_long<true, 32> : (const void*)k_match_long<false, 32>;
            hipError_t e = allow_lds(fn, &configured32[p.counts ? 2 : 1], q.lds_bytes);
            if (e != hipSuccess) return e;
            if (p.counts)
                k_match_long<true, 32><<<grid32, 64, q.lds_bytes, s>>>(q, q.plan, q.feat.f64, q.feat.f32);
            else
                k_match_long<false, 32><<<grid32, 64, q.lds_bytes, s>>>(q, q.plan, q.feat.f64, q.feat.f32);
            return hipGetLastError();
        }
        const void* fn = p.counts ? (const void*)k_match_long<true> : (const void*)k_match_long<false>;
        hipError_t e = allow_lds(fn, &configured[p.counts ? 2 : 3], q.lds_bytes);
        if (e != hipSuccess) return e;
        if (p.counts)
            k_match_long<true><<<grid, 64, q.lds_bytes, s>>>(q, q.plan, q.feat.f64, q.feat.f32);
        else
            k_match_long<false><<<grid, 64, q.lds_bytes, s>>>(q, q.plan, q.feat.f64, q.feat.f32);
        return hipGetLastError();
    }
    if (r32) {
        const void* fn = p.counts ? (const void*)k_match<true, 32> : (const void*)k_match<false, 32>;
        hipError_t e = allow_lds(fn, &configured32[p.counts ? 3 : 0], p.lds_bytes);
        if (e != hipSuccess) return e;
        if (p.counts)
            k_match<true, 32><<<grid32, 64, p.lds_bytes, s>>>(p, p.plan, p.feat.f64, p.feat.f32);
        else
            k_match<false, 32><<<grid32, 64, p.lds_bytes, s>>>(p, p.plan, p.feat.f64, p.feat.f32);
        return hipGetLastError();
    }
    if (p.counts) {
        hipError_t e = allow_lds((const void*)k_match<true>, &configured[0], p.lds_bytes);
        if (e != hipSuccess) return e;
        k_match<true><<<grid, 64, p.lds_bytes, s>>>(p, p.plan, p.feat.f64, p.feat.f32);
    } else {
        hipError_t e = allow_lds((const void*)k_match<false>, &configured[1], p.lds_bytes);
        if (e != hipSuccess) return e;
        k_match<false><<<grid, 64, p.lds_bytes, s>>>(p, p.plan, p.feat.f64, p.feat.f32);
    }
    return hipGetLastError();
}

hipError_t launch_match_persistent(const MatchParams* mps, const uint64_t* prefix, uint32_t n_parts, uint64_t total,
                                   unsigned long long* cursor, uint32_t grab, uint32_t grid, uint32_t lds_bytes,
                                   hipStream_t s) {
    if (total == 0 || grid == 0) return hipSuccess;
    if (total >= (1ull << 60)) return hipErrorInvalidValue;
    static int configured = 0;
    hipError_t e = allow_lds((const void*)k_match_persistent, &configured, lds_bytes);
    if (e != hipSuccess) return e;
    k_match_persistent<<<grid, 64, lds_bytes, s>>>(mps, prefix, n_parts, total, cursor, grab);
    return hipGetLastError();
}

hipError_t launch_match_multi(const MatchParams* mps, const uint64_t* prefix, uint32_t n_parts, uint64_t total,
                              uint32_t lds_bytes, hipStream_t s) {
    if (total == 0) return hipSuccess;
    if (total > kMaxTiles) return hipErrorInvalidValue;   // the grid holds 4 x total workgroups
    static int configured = 0;
    hipError_t e = allow_lds((const void*)k_match_multi, &configured, lds_bytes);
    if (e != hipSuccess) return e;
    k_match_multi<<<(unsigned)((total * 4 + 31) & ~31ull), 64, lds_bytes, s>>>(mps, prefix, n_parts, total);
    return hipGetLastError();
}

hipError_t match_persistent_occupancy(uint32_t lds_bytes, int* blocks_per_cu) {
    static int configured = 0;
    hipError_t e = allow_lds((const void*)k_match_persistent, &configured, lds_bytes);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_match_persistent, 64, lds_bytes);
}

hipError_t launch_zero_bytes(void* p, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const size_t words = n / 16 + 1;
    const unsigned blocks = (unsigned)std::min<size_t>((words + 255) / 256, 4096);
    k_zero_bytes<<<blocks, 256, 0, s>>>((uint8_t*)p, n);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, uint64_t n, unsigned long long v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_fill_u64<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

}  // namespace hb

namespace hb {

hipError_t launch_block_features(const LearnParams& p, hipStream_t s) {
    if (p.n_list == 0 || p.n_spec == 0) return hipSuccess;
    k_block_features<<<p.n_list, 64, 0, s>>>(p);
    return hipGetLastError();
}

hipError_t launch_plan_choice(const PlanChoiceParams& p, hipStream_t s) {
    if (p.n_blocks == 0) return hipSuccess;
    // one wave per 64 blocks: a thread's work is long and serial, so the
    // blocks are spread over as many compute units as they fill
    k_plan_choice<<<(p.n_blocks + 63) / 64, 64, 0, s>>>(p);
    return hipGetLastError();
}

hipError_t launch_log_samples(const LearnParams& p, hipStream_t s) {
    if (p.mp.n_blocks == 0 || p.n_spec == 0 || p.samples == 0) return hipSuccess;
    const uint32_t lds = p.mp.lds_wave_stride;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)k_log_samples, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
        if (e != hipSuccess) return e;
    }
    dim3 grid(p.mp.n_blocks, p.samples);
    k_log_samples<<<grid, 64, lds, s>>>(p);
    return hipGetLastError();
}

}  // namespace hb

namespace hb {

hipError_t launch_pair_log(const PairParams& p, hipStream_t s) {
    if (p.n_spec == 0 || p.samples == 0) return hipSuccess;
    dim3 grid(p.samples, p.n_spec);
    k_pair_log<<<grid, 64, p.lds_bytes, s>>>(p);
    return hipGetLastError();
}

hipError_t launch_pair_features(const PairParams& p, hipStream_t s) {
    const uint64_t rows = (uint64_t)p.n_spec * p.samples;
    if (rows == 0) return hipSuccess;
    k_pair_features<<<(unsigned)((rows + 255) / 256), 256, 0, s>>>(p);
    return hipGetLastError();
}

hipError_t launch_pair_sum(const PairParams& p, hipStream_t s) {
    if (p.n_spec == 0 || p.samples == 0) return hipSuccess;
    k_pair_sum<<<p.n_spec, 256, 0, s>>>(p);
    return hipGetLastError();
}

}  // namespace hb
