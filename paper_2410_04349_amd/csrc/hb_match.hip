// The pair-evaluation kernel of libhb (gfx950).
//
// Work unit: a 64 x 64 tile (i-tile, j-tile) of the upper triangle of one
// block of a key partition.  A workgroup of four waves stages the j-tile's
// attribute values in LDS once; each wave then takes rows i = i0 + w,
// i0 + w + 4, ..., so the pattern tuple t_i is uniform across the wave and
// its 64 lanes hold 64 candidates t_j.  Every lane walks the sequential
// execution path (Section 5.1) for its pair (t_i, t_j): predicates in plan
// order, a reuse bitmap of evaluated / satisfied distinct predicates, a
// rule-end checkpoint that reports a witness (Section 2, "Blocking"), and a
// wave-uniform jump to the checkpoint once no lane can still satisfy the
// current rule.  Matched lanes are compacted with a ballot, one atomic per
// wave-row, and written as packed (min(row) << 32) | max(row).
//
// Edit distance: Myers' bit-parallel algorithm in Hyyro's formulation for
// the Levenshtein distance (pattern = t_i, one bit per pattern byte, the
// pattern-match table built once per row in the wave's LDS), 32-bit for
// patterns <= 32 bytes, 64-bit words with carry chains up to 512 bytes.
// Jaccard: merge intersection of sorted distinct q-gram codes, after the
// exact size filter min(|A|,|B|) * den < num * max(|A|,|B|) => false.
#include "hb_internal.h"

namespace hb {

namespace {

__device__ inline bool bit_valid(const uint8_t* valid, uint32_t r) {
    return valid == nullptr || ((valid[r >> 3] >> (r & 7)) & 1);
}

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
            T sum = a + pv;
            T c1 = sum < a ? 1 : 0;
            T sum2 = sum + carry;
            T c2 = sum2 < sum ? 1 : 0;
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

__device__ inline int myers_dispatch(const uint8_t* peq_bytes, int words, int m,
                                     const uint8_t* text, int n) {
    if (m == 0) return n;
    if (n == 0) return m;
    if (words == 0) return myers<uint32_t, 1>((const uint32_t*)peq_bytes, m, text, n);
    switch (words) {
    case 1: return myers<uint64_t, 1>((const uint64_t*)peq_bytes, m, text, n);
    case 2: return myers<uint64_t, 2>((const uint64_t*)peq_bytes, m, text, n);
    case 3: return myers<uint64_t, 3>((const uint64_t*)peq_bytes, m, text, n);
    case 4: return myers<uint64_t, 4>((const uint64_t*)peq_bytes, m, text, n);
    case 5: return myers<uint64_t, 5>((const uint64_t*)peq_bytes, m, text, n);
    case 6: return myers<uint64_t, 6>((const uint64_t*)peq_bytes, m, text, n);
    case 7: return myers<uint64_t, 7>((const uint64_t*)peq_bytes, m, text, n);
    default: return myers<uint64_t, 8>((const uint64_t*)peq_bytes, m, text, n);
    }
}

// Build the pattern-match table of pattern p (length m) in the wave's LDS.
// words == 0: 32-bit table of 256 entries; else 256 x words 64-bit entries.
__device__ inline void build_peq(uint8_t* peq_bytes, int words, const uint8_t* __restrict__ p, int m,
                                 int lane) {
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
    uint64_t diff = a >= b ? (uint64_t)a - (uint64_t)b : (uint64_t)b - (uint64_t)a;
    return diff <= (uint64_t)d;
}

// tile index -> (block, ti, tj), tiles of a block enumerated column-major
// over the upper triangle: column tj holds ti = 0..tj.
__device__ inline void decode_tile(const MatchParams& P, uint64_t t, uint32_t* b, uint32_t* ti, uint32_t* tj) {
    uint32_t lo = 0, hi = P.n_blocks - 1;
    while (lo < hi) {
        uint32_t mid = (lo + hi + 1) >> 1;
        if (P.tile_prefix[mid] <= t) lo = mid; else hi = mid - 1;
    }
    *b = lo;
    uint64_t u = t - P.tile_prefix[lo];
    uint64_t c = (uint64_t)((sqrt(8.0 * (double)u + 1.0) - 1.0) * 0.5);
    while (c * (c + 1) / 2 > u) --c;
    while ((c + 1) * (c + 2) / 2 <= u) ++c;
    *tj = (uint32_t)c;
    *ti = (uint32_t)(u - c * (c + 1) / 2);
}

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
    const uint32_t* __restrict__ perm = P.perm + bstart;

    // ---------------------------------------------------- stage the j-tile
    int64_t* s_int = (int64_t*)(lds + P.lds_int);
    uint8_t* s_int_valid = lds + P.lds_int_valid;
    for (uint32_t x = tid; x < P.n_int * kTile; x += kThreads) {
        uint32_t res = x / kTile, l = x % kTile;
        int64_t v = 0;
        uint8_t ok = 0;
        if (l < nj) {
            uint32_t row = perm[j0 + l];
            const ColDev& c = P.cols[P.int_attr[res]];
            ok = bit_valid(c.valid, row) ? 1 : 0;
            v = c.values[row];
        }
        s_int[x] = v;
        s_int_valid[x] = ok;
    }
    uint32_t* s_str_len = (uint32_t*)(lds + P.lds_str_len);
    uint8_t* s_str_valid = lds + P.lds_str_valid;
    for (uint32_t res = 0; res < P.n_str; ++res) {
        const ColDev& c = P.cols[P.str_attr[res]];
        uint8_t* dst = lds + P.lds_str[res];
        const uint32_t stride = P.str_stride[res];
        const bool staged = !((P.str_global >> res) & 1);
        for (uint32_t l = wave; l < kTile; l += kWaves) {
            uint32_t len = 0;
            uint8_t ok = 0;
            if (l < nj) {
                uint32_t row = perm[j0 + l];
                ok = bit_valid(c.valid, row) ? 1 : 0;
                uint64_t o = c.off[row];
                len = (uint32_t)(c.off[row + 1] - o);
                if (staged)
                    for (uint32_t x = lane; x < len; x += 64) dst[l * stride + x] = c.bytes[o + x];
            }
            if (lane == 0) {
                s_str_len[res * kTile + l] = len;
                s_str_valid[res * kTile + l] = ok;
            }
        }
    }
    uint32_t* s_gram_cnt = (uint32_t*)(lds + P.lds_gram_cnt);
    uint8_t* s_gram_flag = lds + P.lds_gram_flag;
    for (uint32_t res = 0; res < P.n_gram; ++res) {
        const GramDev& g = P.gram[res];
        const ColDev& c = P.cols[g.attr];
        uint32_t* dst = (uint32_t*)(lds + P.lds_gram[res]);
        const bool staged = !((P.gram_global >> res) & 1);
        for (uint32_t l = wave; l < kTile; l += kWaves) {
            uint32_t cnt = 0;
            uint8_t fl = 0;
            if (l < nj) {
                uint32_t row = perm[j0 + l];
                if (bit_valid(c.valid, row)) {
                    cnt = g.cnt[row];
                    fl = (uint8_t)(2 | (g.flags[row] & 1));
                    const uint32_t* src = g.codes + g.off[row];
                    if (staged)
                        for (uint32_t x = lane; x < cnt; x += 64) dst[l * g.max_cnt + x] = src[x];
                }
            }
            if (lane == 0) {
                s_gram_cnt[res * kTile + l] = cnt;
                s_gram_flag[res * kTile + l] = fl;
            }
        }
    }
    __syncthreads();

    const uint32_t row_j = lane < (int)nj ? perm[j0 + lane] : 0;
    uint8_t* wbase = lds + P.lds_wave_base + wave * P.lds_wave_stride;
    uint8_t* peq = wbase + P.lds_wave_peq;
    unsigned long long* counter = P.counter;

    for (uint32_t ii = wave; ii < ni; ii += kWaves) {
        const uint32_t l = lane;
        const bool lane_pair = (l < nj) && (!diag || l > ii);
        if (!__any(lane_pair)) continue;
        const uint32_t row_i = perm[i0 + ii];

        // canonical owner: a pair agreeing on an earlier key was evaluated there
        bool alive_pair = lane_pair;
        for (uint32_t k = 0; k < P.n_prev; ++k) {
            const uint32_t res = P.prev_res[k];
            const ColDev& c = P.cols[P.int_attr[res]];
            const bool iv = bit_valid(c.valid, row_i);
            const int64_t vi = c.values[row_i];
            if (iv && s_int_valid[res * kTile + l] && s_int[res * kTile + l] == vi) alive_pair = false;
        }

        uint64_t evaluated = 0, result = 0;
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
            const Instr ins = P.plan[pc];
            if (ins.op == OP_CP) {
                matched = matched || alive;
                alive = alive_pair && !matched;
                if (!__any(alive)) {
                    // every lane is matched or has no pair: the rest is moot
                    if (!__any(alive_pair && !matched)) break;
                }
                ++pc;
                continue;
            }
            if (!__any(alive)) { pc = ins.cp; continue; }
            const uint64_t bit = 1ull << ins.slot;
            const bool need = alive && !(evaluated & bit);
            if (__any(need)) {
                bool r = false;
                const uint32_t res = ins.res;
                switch (ins.op) {
                case OP_EQ_INT:
                case OP_ABSDIFF: {
                    const ColDev& c = P.cols[P.int_attr[res]];
                    const bool iv = bit_valid(c.valid, row_i);
                    const int64_t vi = c.values[row_i];
                    if (need) {
                        const bool jv = s_int_valid[res * kTile + l] != 0;
                        const int64_t vj = s_int[res * kTile + l];
                        r = iv && jv && (ins.op == OP_EQ_INT ? vi == vj : absdiff_le(vi, vj, ins.k_or_d));
                    }
                    break;
                }
                case OP_EQ_STR: {
                    const ColDev& c = P.cols[P.str_attr[res]];
                    const bool iv = bit_valid(c.valid, row_i);
                    const uint64_t o = c.off[row_i];
                    const uint32_t m = (uint32_t)(c.off[row_i + 1] - o);
                    const uint8_t* si = c.bytes + o;
                    if (need) {
                        const uint32_t n = s_str_len[res * kTile + l];
                        bool eq = iv && s_str_valid[res * kTile + l] && m == n;
                        if ((P.str_global >> res) & 1) {
                            const uint8_t* sj = c.bytes + c.off[row_j];
                            for (uint32_t x = 0; eq && x < m; ++x) eq = si[x] == sj[x];
                        } else {
                            const uint8_t* sj = lds + P.lds_str[res] + l * P.str_stride[res];
                            for (uint32_t x = 0; eq && x < m; ++x) eq = si[x] == sj[x];
                        }
                        r = eq;
                    }
                    break;
                }
                case OP_ED: {
                    const ColDev& c = P.cols[P.str_attr[res]];
                    const bool iv = bit_valid(c.valid, row_i);
                    const uint64_t o = c.off[row_i];
                    const int m = (int)(c.off[row_i + 1] - o);
                    const int k = (int)ins.k_or_d;
                    const int words = m <= 32 ? 0 : (m + 63) / 64;
                    int cached = -1;
#pragma unroll
                    for (int s = 0; s < kMaxStrRes; ++s) if (s == (int)res) cached = ed_cache[s];
                    const int n = (int)s_str_len[res * kTile + l];
                    const bool jv = s_str_valid[res * kTile + l] != 0;
                    const bool run = need && iv && jv && cached < 0 && abs(m - n) <= k;
                    if (iv && __any(run) && peq_res != (int)res) {
                        build_peq(peq, words, c.bytes + o, m, lane);
                        peq_res = (int)res;
                    }
                    if (need) {
                        int dist = cached;
                        if (run) {
                            if ((P.str_global >> res) & 1)
                                dist = myers_dispatch(peq, words, m, c.bytes + c.off[row_j], n);
                            else
                                dist = myers_dispatch(peq, words, m, lds + P.lds_str[res] + l * P.str_stride[res], n);
#pragma unroll
                            for (int s = 0; s < kMaxStrRes; ++s) if (s == (int)res) ed_cache[s] = dist;
                        }
                        r = iv && jv && abs(m - n) <= k && dist >= 0 && dist <= k;
                    }
                    break;
                }
                case OP_JAC: {
                    const GramDev& g = P.gram[res];
                    const ColDev& c = P.cols[g.attr];
                    const bool iv = bit_valid(c.valid, row_i);
                    const uint32_t ca = iv ? g.cnt[row_i] : 0;
                    const bool ishort = iv && (g.flags[row_i] & 1);
                    uint32_t* ig = (uint32_t*)(wbase + P.lds_wave_igram[res]);
                    if (iv && !(igram_loaded & (1u << res))) {
                        const uint32_t* src = g.codes + g.off[row_i];
                        for (uint32_t x = lane; x < ca; x += 64) ig[x] = src[x];
                        wave_sync();
                        igram_loaded |= 1u << res;
                    }
                    if (need) {
                        const uint8_t fl = s_gram_flag[res * kTile + l];
                        const bool jv = (fl & 2) != 0;
                        if (iv && jv) {
                            const uint32_t cb = s_gram_cnt[res * kTile + l];
                            const bool jshort = (fl & 1) != 0;
                            const uint64_t num = ins.num, den = ins.den;
                            const uint32_t mn = min(ca, cb), mx = max(ca, cb);
                            if ((uint64_t)mn * den < num * (uint64_t)mx) {
                                r = false;
                            } else {
                                int cached = -1;
#pragma unroll
                                for (int s = 0; s < kMaxGramRes; ++s) if (s == (int)res) cached = jac_cache[s];
                                uint32_t I;
                                if (cached >= 0) {
                                    I = (uint32_t)cached;
                                } else if ((P.gram_global >> res) & 1) {
                                    I = intersect(ig, ca, ishort, g.codes + g.off[row_j], cb, jshort);
                                } else {
                                    I = intersect(ig, ca, ishort,
                                                  (const uint32_t*)(lds + P.lds_gram[res]) + l * g.max_cnt, cb, jshort);
                                }
                                {
#pragma unroll
                                    for (int s = 0; s < kMaxGramRes; ++s) if (s == (int)res) jac_cache[s] = (int)I;
                                }
                                const uint64_t U = (uint64_t)ca + cb - I;
                                r = (U == 0) || ((uint64_t)I * den >= num * U);
                            }
                        }
                    }
                    break;
                }
                default:
                    break;
                }
                if (need) {
                    evaluated |= bit;
                    if (r) result |= bit;
                }
            }
            alive = alive && ((result & bit) != 0);
            ++pc;
        }

        // ballot compaction of matched pairs
        const uint64_t mask = __ballot(matched);
        if (mask) {
            const uint32_t cnt = __popcll(mask);
            unsigned long long basev = 0;
            if (lane == 0) basev = atomicAdd(counter, (unsigned long long)cnt);
            basev = __shfl(basev, 0);
            if (matched) {
                const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
                const uint64_t pos = basev + __popcll(mask & lt);
                if (pos < P.cap) {
                    const uint32_t row_j = perm[j0 + l];
                    const uint64_t a = row_i < row_j ? row_i : row_j;
                    const uint64_t c = row_i < row_j ? row_j : row_i;
                    P.out[pos] = (a << 32) | c;
                }
            }
        }
    }
}

}  // namespace

hipError_t launch_match(const MatchParams& p, hipStream_t s) {
    if (p.n_tiles == 0) return hipSuccess;
    static int configured = 0;
    if (p.lds_bytes > 65536 && configured < (int)p.lds_bytes) {
        hipError_t e = hipFuncSetAttribute((const void*)k_match, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)p.lds_bytes);
        if (e != hipSuccess) return e;
        configured = (int)p.lds_bytes;
    }
    k_match<<<(unsigned)p.n_tiles, kThreads, p.lds_bytes, s>>>(p);
    return hipGetLastError();
}

}  // namespace hb
