// The pair-evaluation kernel of libhb (gfx950).
//
// Work unit: a 64 x 64 tile (i-tile, j-tile) of the upper triangle of one
// block of a key partition.  A workgroup of four waves stages the j-tile's
// compact feature columns (values, lengths, set sizes, signatures) in LDS
// once; each wave then takes rows i = i0 + w, i0 + w + 4, ..., so tuple t_i
// is uniform across the wave and its 64 lanes hold 64 candidates t_j.
//
// Every lane walks the sequential execution path (Section 5.1) for its pair
// (t_i, t_j): steps in plan order, a reuse bitmap of evaluated / satisfied
// steps, a rule-end checkpoint that reports a witness (Section 2,
// "Blocking"), and a wave-uniform jump to the checkpoint once no lane can
// still satisfy the current rule.  Within a rule the plan runs exact,
// cheap necessary-condition filters before the expensive predicates
// (edit distance, Jaccard, string equality), so the expensive code runs for
// a wave only when some lane passed all of the rule's filters.  Matched lanes
// are compacted with a ballot, one atomic per wave-row.
//
// Edit distance: Myers' bit-parallel algorithm in Hyyro's formulation for
// the Levenshtein distance (pattern = t_i, one bit per pattern byte, the
// pattern-match table built once per row in the wave's LDS), 32-bit words
// for patterns <= 32 bytes, 64-bit words with carry chains up to 256 bytes.
// Jaccard: merge intersection of the sorted distinct q-gram codes.
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
    for (int pos = 0; pos < n; ++pos) {
        const T* eq = peq + (uint32_t)text[pos] * W;
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

__device__ inline int myers_dispatch(const uint8_t* peq_bytes, int words, int m, const uint8_t* text, int n) {
    if (m == 0) return n;
    if (n == 0) return m;
    if (words == 0) return myers<uint32_t, 1>((const uint32_t*)peq_bytes, m, text, n);
    switch (words) {
    case 1: return myers<uint64_t, 1>((const uint64_t*)peq_bytes, m, text, n);
    case 2: return myers<uint64_t, 2>((const uint64_t*)peq_bytes, m, text, n);
    case 3: return myers<uint64_t, 3>((const uint64_t*)peq_bytes, m, text, n);
    default: return myers<uint64_t, 4>((const uint64_t*)peq_bytes, m, text, n);
    }
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
__device__ inline uint32_t intersect(const uint32_t* __restrict__ A, uint32_t ca, bool ashort,
                                     const uint32_t* __restrict__ B, uint32_t cb, bool bshort) {
    if (ashort || bshort) return (ashort && bshort && A[0] == B[0]) ? 1u : 0u;
    uint32_t ia = 0, ib = 0, I = 0;
    while (ia < ca && ib < cb) {
        const uint32_t x = A[ia], y = B[ib];
        I += x == y ? 1u : 0u;
        ia += x <= y ? 1u : 0u;
        ib += y <= x ? 1u : 0u;
    }
    return I;
}

__device__ inline bool absdiff_le(int64_t a, int64_t b, int64_t d) {
    const uint64_t diff = a >= b ? (uint64_t)a - (uint64_t)b : (uint64_t)b - (uint64_t)a;
    return diff <= (uint64_t)d;
}

// tile index -> (block, ti, tj), tiles of a block enumerated column-major
// over the upper triangle: column tj holds ti = 0..tj.
__device__ inline void decode_tile(const MatchParams& P, uint64_t t, uint32_t* b, uint32_t* ti, uint32_t* tj) {
    uint32_t lo = 0, hi = P.n_blocks - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (P.tile_prefix[mid] <= t) lo = mid; else hi = mid - 1;
    }
    *b = lo;
    const uint64_t u = t - P.tile_prefix[lo];
    uint64_t c = (uint64_t)((sqrt(8.0 * (double)u + 1.0) - 1.0) * 0.5);
    while (c * (c + 1) / 2 > u) --c;
    while ((c + 1) * (c + 2) / 2 <= u) ++c;
    *tj = (uint32_t)c;
    *ti = (uint32_t)(u - c * (c + 1) / 2);
}

template <int N>
__device__ inline int pick(const int (&a)[N], int i) {
    int v = -1;
#pragma unroll
    for (int s = 0; s < N; ++s) if (s == i) v = a[s];
    return v;
}

template <int N>
__device__ inline void put(int (&a)[N], int i, int v) {
#pragma unroll
    for (int s = 0; s < N; ++s) if (s == i) a[s] = v;
}

template <bool kCount>
__global__ __launch_bounds__(kThreads) void k_match(const MatchParams P) {
    extern __shared__ __align__(16) uint8_t lds[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    // XCD-aware remap: consecutive workgroups go round-robin to the 8 XCDs;
    // give each XCD a contiguous range of tiles so a block's tiles share L2.
    const uint64_t G = gridDim.x;
    const uint64_t bid = blockIdx.x;
    const uint64_t xcd = bid & 7, idx = bid >> 3;
    const uint64_t q8 = G >> 3, r8 = G & 7;
    const uint64_t t = xcd * q8 + (xcd < r8 ? xcd : r8) + idx;
    if (t >= P.n_tiles) return;

    uint32_t b, ti, tj;
    decode_tile(P, t, &b, &ti, &tj);
    const uint32_t bstart = P.blk_start[b], bsize = P.blk_size[b];
    const uint32_t i0 = ti * kTile, j0 = tj * kTile;
    const uint32_t ni = min((uint32_t)kTile, bsize - i0), nj = min((uint32_t)kTile, bsize - j0);
    const bool diag = ti == tj;

    const uint64_t n = P.feat.n;
    const uint64_t* __restrict__ f64 = P.feat.f64;
    const uint32_t* __restrict__ f32 = P.feat.f32;
    const uint32_t n64 = P.n_int + P.n_str + P.n_gram;
    const uint32_t n32 = 2 + P.n_str + P.n_gram;
    const uint32_t str64 = P.n_int, gram64 = P.n_int + P.n_str;    // first f64 column of each kind
    const uint32_t str32 = 2, gram32 = 2 + P.n_str;                 // first f32 column of each kind

    // ------------------------------------- stage the plan, i-tile and j-tile
    Instr* s_plan = (Instr*)(lds + P.lds_plan);
    for (uint32_t x = tid; x < P.plan_len; x += kThreads) s_plan[x] = P.plan[x];
    uint64_t* s64 = (uint64_t*)(lds + P.lds_f64);
    uint32_t* s32 = (uint32_t*)(lds + P.lds_f32);
    uint64_t* i64 = (uint64_t*)(lds + P.lds_i64);
    uint32_t* i32 = (uint32_t*)(lds + P.lds_i32);
    const uint64_t pj = (uint64_t)bstart + j0, pi0 = (uint64_t)bstart + i0;
    for (uint32_t x = tid; x < n64 * kTile; x += kThreads) {
        const uint32_t f = x / kTile, l = x % kTile;
        s64[x] = l < nj ? f64[f * n + pj + l] : 0ull;
        i64[x] = l < ni ? f64[f * n + pi0 + l] : 0ull;
    }
    for (uint32_t x = tid; x < n32 * kTile; x += kThreads) {
        const uint32_t f = x / kTile, l = x % kTile;
        s32[x] = l < nj ? f32[f * n + pj + l] : 0u;
        i32[x] = l < ni ? f32[f * n + pi0 + l] : 0u;
    }
    unsigned long long* s_cnt = (unsigned long long*)(lds + P.lds_counts);
    if constexpr (kCount)
        for (uint32_t x = tid; x < P.plan_len * 4 + 1; x += kThreads) s_cnt[x] = 0;
    __syncthreads();

    const uint32_t row_j = s32[lane];
    const uint32_t vmask_j = s32[kTile + lane];
    uint8_t* wbase = lds + P.lds_wave_base + wave * P.lds_wave_stride;
    uint8_t* peq = wbase + P.lds_wave_peq;

    for (uint32_t ii = wave; ii < ni; ii += kWaves) {
        const bool lane_pair = ((uint32_t)lane < nj) && (!diag || (uint32_t)lane > ii);
        if (!__any(lane_pair)) continue;
        // t_i's features: uniform LDS reads, moved to scalar registers
        auto I64 = [&](uint32_t f) -> uint64_t {
            const uint64_t v = i64[f * kTile + ii];
            return ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32)) << 32) |
                   (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)v);
        };
        auto I32 = [&](uint32_t f) -> uint32_t { return __builtin_amdgcn_readfirstlane(i32[f * kTile + ii]); };
        const uint32_t row_i = I32(0);
        const uint32_t vmask_i = I32(1);
        const uint32_t vboth = vmask_i & vmask_j;

        // canonical owner: a pair agreeing on an earlier key was evaluated there
        bool alive_pair = lane_pair;
        for (uint32_t k = 0; k < P.n_prev; ++k) {
            const uint32_t res = P.prev_res[k];
            if (((vboth >> res) & 1) && I64(res) == s64[res * kTile + lane]) alive_pair = false;
        }
        if constexpr (kCount) {
            const uint64_t pb = __ballot(alive_pair);
            if (lane == 0 && pb) atomicAdd(&s_cnt[P.plan_len * 4], (unsigned long long)__popcll(pb));
        }

        uint64_t ev0 = 0, ev1 = 0, rs0 = 0, rs1 = 0;
        bool matched = false;
        bool alive = alive_pair;
        int peq_res = -1;
        uint32_t igram_loaded = 0;
        int ed_cache[kMaxStrRes];
        int jac_cache[kMaxGramRes];
#pragma unroll
        for (int s = 0; s < kMaxStrRes; ++s) ed_cache[s] = -1;
#pragma unroll
        for (int s = 0; s < kMaxGramRes; ++s) jac_cache[s] = -1;

        uint32_t pc = 0;
        while (pc < P.plan_len) {
            Instr ins;
            {
                const uint4 raw = *(const uint4*)&s_plan[pc];
                const uint32_t w0 = __builtin_amdgcn_readfirstlane(raw.x);
                const uint32_t w1 = __builtin_amdgcn_readfirstlane(raw.y);
                const uint32_t w2 = __builtin_amdgcn_readfirstlane(raw.z);
                const uint32_t w3 = __builtin_amdgcn_readfirstlane(raw.w);
                ins.op = (uint8_t)w0;
                ins.slot = (uint8_t)(w0 >> 8);
                ins.res = (uint8_t)(w0 >> 16);
                ins.cp = (uint16_t)w1;
                ins.param = ((uint64_t)w3 << 32) | w2;
            }
            if (ins.op == OP_CP) {
                matched = matched || alive;
                alive = alive_pair && !matched;
                if (!__any(alive)) break;   // every lane is matched or has no pair
                ++pc;
                continue;
            }
            if (!__any(alive)) { pc = ins.cp; continue; }
            const bool hi = ins.slot >= 64;
            const uint64_t bit = 1ull << (ins.slot & 63);
            const bool done = ((hi ? ev1 : ev0) & bit) != 0;
            const bool need = alive && !done;
            if (__any(need)) {
                bool r = false;
                uint32_t work = 1;
                const uint32_t res = ins.res;
                switch (ins.op) {
                case OP_EQ_INT:
                case OP_ABSDIFF: {
                    const int64_t vi = (int64_t)I64(res);
                    const int64_t vj = (int64_t)s64[res * kTile + lane];
                    const bool v = (vboth >> res) & 1;
                    r = v && (ins.op == OP_EQ_INT ? vi == vj : absdiff_le(vi, vj, (int64_t)ins.param));
                    break;
                }
                case OP_EQF:
                case OP_EDF: {
                    const bool v = (vboth >> (16 + res)) & 1;
                    const uint32_t li = I32(str32 + res);
                    const uint32_t lj = s32[(str32 + res) * kTile + lane];
                    const uint64_t ci = I64(str64 + res);
                    const uint64_t cj = s64[(str64 + res) * kTile + lane];
                    if (ins.op == OP_EQF) {
                        r = v && li == lj && ci == cj;
                    } else {
                        const int k = (int)ins.param;
                        const int d1 = __popcll(ci & ~cj), d2 = __popcll(cj & ~ci);
                        r = v && abs((int)li - (int)lj) <= k && max(d1, d2) <= k;
                    }
                    break;
                }
                case OP_JACF: {
                    const bool v = (vboth >> (24 + res)) & 1;
                    const uint64_t sa = I32(gram32 + res) & 0x7FFFFFFFu;
                    const uint64_t sb = s32[(gram32 + res) * kTile + lane] & 0x7FFFFFFFu;
                    const uint64_t gi = I64(gram64 + res);
                    const uint64_t gj = s64[(gram64 + res) * kTile + lane];
                    const uint64_t ua = sa - (uint64_t)__popcll(gi & ~gj);
                    const uint64_t ub = sb - (uint64_t)__popcll(gj & ~gi);
                    const uint64_t iub = ua < ub ? ua : ub;
                    const uint64_t num = ins.param >> 32, den = ins.param & 0xFFFFFFFFu;
                    r = v && iub * (num + den) >= num * (sa + sb);
                    break;
                }
                case OP_EQ_STR: {
                    const ColDev& c = P.cols[P.str_attr[res]];
                    const bool v = (vboth >> (16 + res)) & 1;
                    const uint32_t li = I32(str32 + res);
                    const uint32_t lj = s32[(str32 + res) * kTile + lane];
                    const uint8_t* si = c.bytes + c.off[row_i];
                    if (need) {
                        bool eq = v && li == lj;
                        work = 0;
                        if (eq) {
                            const uint8_t* sj = c.bytes + c.off[row_j];
                            work = li;
                            for (uint32_t x = 0; eq && x < li; ++x) eq = si[x] == sj[x];
                        }
                        r = eq;
                    }
                    break;
                }
                case OP_ED: {
                    const ColDev& c = P.cols[P.str_attr[res]];
                    const bool iv = (vmask_i >> (16 + res)) & 1;
                    const bool v = (vboth >> (16 + res)) & 1;
                    const int m = (int)I32(str32 + res);
                    const int nn = (int)s32[(str32 + res) * kTile + lane];
                    const int k = (int)ins.param;
                    const int words = m <= 32 ? 0 : (m + 63) / 64;
                    const int cached = pick(ed_cache, (int)res);
                    const bool run = need && v && cached < 0 && abs(m - nn) <= k;
                    if (iv && peq_res != (int)res && __any(run)) {
                        build_peq(peq, words, c.bytes + c.off[row_i], m, lane);
                        peq_res = (int)res;
                    }
                    if (need) {
                        int dist = cached;
                        work = run ? (uint32_t)nn * (uint32_t)max(1, (m + 31) / 32) : 0u;
                        if (run) {
                            dist = myers_dispatch(peq, words, m, c.bytes + c.off[row_j], nn);
                            put(ed_cache, (int)res, dist);
                        }
                        r = v && abs(m - nn) <= k && dist >= 0 && dist <= k;
                    }
                    break;
                }
                case OP_JAC: {
                    const GramDev& g = P.gram[res];
                    const bool iv = (vmask_i >> (24 + res)) & 1;
                    const bool v = (vboth >> (24 + res)) & 1;
                    const uint32_t ia = I32(gram32 + res);
                    const uint32_t ca = ia & 0x7FFFFFFFu;
                    const bool ishort = (ia >> 31) != 0;
                    uint32_t* ig = (uint32_t*)(wbase + P.lds_wave_igram[res]);
                    if (iv && !((igram_loaded >> res) & 1)) {
                        const uint32_t* src = g.codes + g.off[row_i];
                        for (uint32_t x = lane; x < ca; x += 64) ig[x] = src[x];
                        wave_sync();
                        igram_loaded |= 1u << res;
                    }
                    if (need && v) {
                        const uint32_t jb = s32[(gram32 + res) * kTile + lane];
                        const uint32_t cb = jb & 0x7FFFFFFFu;
                        const bool jshort = (jb >> 31) != 0;
                        int I = pick(jac_cache, (int)res);
                        work = I < 0 ? ca + cb : 0u;
                        if (I < 0) {
                            I = (int)intersect(ig, ca, ishort, g.codes + g.off[row_j], cb, jshort);
                            put(jac_cache, (int)res, I);
                        }
                        const uint64_t U = (uint64_t)ca + cb - (uint64_t)I;
                        r = (U == 0) || ((uint64_t)I * (ins.param & 0xFFFFFFFFu) >= (ins.param >> 32) * U);
                    }
                    break;
                }
                default:
                    break;
                }
                if (need) {
                    if (hi) { ev1 |= bit; if (r) rs1 |= bit; }
                    else { ev0 |= bit; if (r) rs0 |= bit; }
                }
                if constexpr (kCount) {
                    const uint64_t nb = __ballot(need), rb = __ballot(need && r);
                    uint32_t w = need ? work : 0u;
                    for (int o = 32; o > 0; o >>= 1) w += __shfl_xor(w, o);
                    if (lane == 0) {
                        atomicAdd(&s_cnt[pc * 4 + 0], 1ull);
                        atomicAdd(&s_cnt[pc * 4 + 1], (unsigned long long)__popcll(nb));
                        atomicAdd(&s_cnt[pc * 4 + 2], (unsigned long long)__popcll(rb));
                        atomicAdd(&s_cnt[pc * 4 + 3], (unsigned long long)w);
                    }
                }
            }
            alive = alive && (((hi ? rs1 : rs0) & bit) != 0);
            ++pc;
        }

        // ballot compaction of matched pairs
        const uint64_t mask = __ballot(matched);
        if (mask) {
            const uint32_t cnt = __popcll(mask);
            unsigned long long basev = 0;
            if (lane == 0) basev = atomicAdd(P.counter, (unsigned long long)cnt);
            basev = __shfl(basev, 0);
            if (matched) {
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
        for (uint32_t x = tid; x < P.plan_len * 4 + 1; x += kThreads)
            if (s_cnt[x]) atomicAdd(&P.counts[x], s_cnt[x]);
    }
}

}  // namespace

hipError_t launch_match(const MatchParams& p, hipStream_t s) {
    if (p.n_tiles == 0) return hipSuccess;
    const void* fn = p.counts ? (const void*)k_match<true> : (const void*)k_match<false>;
    static int configured[2] = {0, 0};
    int& cfg = configured[p.counts ? 1 : 0];
    if (p.lds_bytes > 65536 && cfg < (int)p.lds_bytes) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds_bytes);
        if (e != hipSuccess) return e;
        cfg = (int)p.lds_bytes;
    }
    if (p.counts)
        k_match<true><<<(unsigned)p.n_tiles, kThreads, p.lds_bytes, s>>>(p);
    else
        k_match<false><<<(unsigned)p.n_tiles, kThreads, p.lds_bytes, s>>>(p);
    return hipGetLastError();
}

}  // namespace hb
