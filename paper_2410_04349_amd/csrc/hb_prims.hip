// Streaming primitives of libhb for gfx950: column statistics, scans, a
// stable LSD radix sort, partition (grouping by exact key value) helpers,
// the q-gram index build and the LSH histograms behind the selectivity
// estimate of Section 4.2.  All are HBM-bound streaming kernels.
#include "hb_internal.h"

namespace hb {

namespace {

constexpr int kBlock = 256;

__device__ inline bool bit_valid(const uint8_t* valid, uint32_t r) {
    return valid == nullptr || ((valid[r >> 3] >> (r & 7)) & 1);
}

__device__ inline uint64_t order_key(int64_t v) { return (uint64_t)v ^ 0x8000000000000000ull; }

// splitmix64 output function (Steele, Lea and Flood, OOPSLA 2014)
__device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// ------------------------------------------------------------ column stats

__global__ void k_string_stats(const uint64_t* __restrict__ off, uint32_t n, uint32_t* max_len,
                               unsigned long long* total, uint32_t* bad) {
    uint32_t local_max = 0;
    unsigned long long local_sum = 0;
    uint32_t local_bad = 0;
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        uint64_t a = off[r], b = off[r + 1];
        if (b < a) { local_bad = 1; continue; }
        uint64_t L = b - a;
        if (L > 0xFFFFFFFFull) { local_bad = 1; continue; }
        local_max = max(local_max, (uint32_t)L);
        local_sum += L;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && off[0] != 0) local_bad = 1;
    // wave, then workgroup reduction: one set of atomics per workgroup (the
    // grid is a few hundred workgroups; atomics on one address serialise)
    __shared__ uint32_t s_max[kBlock / 64], s_bad[kBlock / 64];
    __shared__ unsigned long long s_sum[kBlock / 64];
    for (int o = 32; o > 0; o >>= 1) {
        local_max = max(local_max, (uint32_t)__shfl_xor((int)local_max, o));
        local_sum += __shfl_xor(local_sum, o);
        local_bad |= (uint32_t)__shfl_xor((int)local_bad, o);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_max[w] = local_max;
        s_sum[w] = local_sum;
        s_bad[w] = local_bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int x = 1; x < kBlock / 64; ++x) {
            local_max = max(local_max, s_max[x]);
            local_sum += s_sum[x];
            local_bad |= s_bad[x];
        }
        atomicMax(max_len, local_max);
        atomicAdd(total, local_sum);
        if (local_bad) atomicOr(bad, 1u);
    }
}

__global__ void k_minmax(const int64_t* __restrict__ vals, const uint8_t* __restrict__ valid, uint32_t n,
                         unsigned long long* mn, unsigned long long* mx, unsigned int* nvalid) {
    unsigned long long lmin = ~0ull, lmax = 0;
    unsigned int cnt = 0;
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        if (!bit_valid(valid, r)) continue;
        unsigned long long k = order_key(vals[r]);
        lmin = min(lmin, k);
        lmax = max(lmax, k);
        ++cnt;
    }
    for (int o = 32; o > 0; o >>= 1) {
        lmin = min(lmin, (unsigned long long)__shfl_xor(lmin, o));
        lmax = max(lmax, (unsigned long long)__shfl_xor(lmax, o));
        cnt += (unsigned int)__shfl_xor((int)cnt, o);
    }
    __shared__ unsigned long long s_min[kBlock / 64], s_max[kBlock / 64];
    __shared__ unsigned int s_cnt[kBlock / 64];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_min[w] = lmin;
        s_max[w] = lmax;
        s_cnt[w] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int x = 1; x < kBlock / 64; ++x) {
            lmin = min(lmin, s_min[x]);
            lmax = max(lmax, s_max[x]);
            cnt += s_cnt[x];
        }
        atomicMin(mn, lmin);
        atomicMax(mx, lmax);
        atomicAdd(nvalid, cnt);
    }
}

// ------------------------------------------------------------ scan
// Exclusive scan in three phases: per-chunk totals, scan of the totals
// (recursively), per-chunk scan with the chunk's prefix.

constexpr int kScanItems = 8;
constexpr size_t kScanChunk = (size_t)kBlock * kScanItems;

template <typename T>
__device__ T block_exclusive_scan(T v, T* smem, T* total) {
    // smem: kBlock / 64 entries
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    T x = v;
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) smem[wave] = x;
    __syncthreads();
    T wprefix = 0, all = 0;
    for (int w = 0; w < kBlock / 64; ++w) {
        T t = smem[w];
        if (w < wave) wprefix += t;
        all += t;
    }
    __syncthreads();
    *total = all;
    return wprefix + x - v;
}

template <typename T>
__global__ void k_scan_reduce(const T* __restrict__ in, size_t n, T* __restrict__ partial) {
    __shared__ T smem[kBlock / 64];
    size_t base = (size_t)blockIdx.x * kScanChunk;
    T s = 0;
    for (int it = 0; it < kScanItems; ++it) {
        size_t idx = base + (size_t)threadIdx.x * kScanItems + it;
        if (idx < n) s += in[idx];
    }
    T total;
    block_exclusive_scan<T>(s, smem, &total);
    if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

template <typename T>
__global__ void k_scan_final(const T* __restrict__ in, size_t n, const T* __restrict__ prefix,
                             T* __restrict__ out) {
    __shared__ T smem[kBlock / 64];
    size_t base = (size_t)blockIdx.x * kScanChunk;
    T vals[kScanItems];
    T s = 0;
    for (int it = 0; it < kScanItems; ++it) {
        size_t idx = base + (size_t)threadIdx.x * kScanItems + it;
        vals[it] = idx < n ? in[idx] : (T)0;
        s += vals[it];
    }
    T total;
    T ex = block_exclusive_scan<T>(s, smem, &total);
    T run = ex + (prefix ? prefix[blockIdx.x] : (T)0);
    for (int it = 0; it < kScanItems; ++it) {
        size_t idx = base + (size_t)threadIdx.x * kScanItems + it;
        if (idx < n) out[idx] = run;
        run += vals[it];
    }
}

template <typename T>
hipError_t scan_impl(const T* in, T* out, size_t n, T* tmp, hipStream_t s) {
    if (n == 0) return hipSuccess;
    size_t blocks = (n + kScanChunk - 1) / kScanChunk;
    if (blocks == 1) {
        k_scan_final<T><<<1, kBlock, 0, s>>>(in, n, nullptr, out);
        return hipGetLastError();
    }
    T* partial = tmp;
    T* rest = tmp + blocks;
    k_scan_reduce<T><<<(unsigned)blocks, kBlock, 0, s>>>(in, n, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = scan_impl<T>(partial, partial, blocks, rest, s);
    if (e != hipSuccess) return e;
    k_scan_final<T><<<(unsigned)blocks, kBlock, 0, s>>>(in, n, partial, out);
    return hipGetLastError();
}

// ------------------------------------------------------------ radix sort

constexpr int kRsItems = 16;
constexpr uint32_t kRsChunk = kBlock * kRsItems;

__global__ void k_rs_hist(const uint64_t* __restrict__ keys, uint32_t n, int shift,
                          uint32_t* __restrict__ hist, uint32_t G) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    uint32_t base = blockIdx.x * kRsChunk;
    for (int it = 0; it < kRsItems; ++it) {
        uint32_t idx = base + it * kBlock + threadIdx.x;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 255], 1u);
    }
    __syncthreads();
    hist[(size_t)threadIdx.x * G + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: elements of a chunk are ranked in (round, wave, lane)
// order, which is their order in memory.
__global__ void k_rs_scatter(const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                             uint64_t* __restrict__ kout, uint32_t* __restrict__ vout, uint32_t n,
                             int shift, const uint32_t* __restrict__ offs, uint32_t G) {
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[kBlock / 64][256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    base[tid] = offs[(size_t)tid * G + blockIdx.x];
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int it = 0; it < kRsItems; ++it) {
        for (int w = 0; w < kBlock / 64; ++w) wcnt[w][tid] = 0;
        __syncthreads();
        uint32_t idx = blockIdx.x * kRsChunk + it * kBlock + tid;
        bool act = idx < n;
        uint64_t key = act ? kin[idx] : 0;
        uint32_t val = (act && vin) ? vin[idx] : 0;
        uint32_t d = (uint32_t)((key >> shift) & 255);
        uint64_t peers = __ballot(act);
        for (int b = 0; b < 8; ++b) {
            uint64_t bb = __ballot((d >> b) & 1);
            peers &= ((d >> b) & 1) ? bb : ~bb;
        }
        uint32_t rank = __popcll(peers & lt_mask);
        if (act && rank == 0) wcnt[wave][d] = __popcll(peers);
        __syncthreads();
        if (act) {
            uint32_t o = base[d] + rank;
            for (int w = 0; w < wave; ++w) o += wcnt[w][d];
            kout[o] = key;
            if (vout) vout[o] = val;
        }
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < kBlock / 64; ++w) add += wcnt[w][tid];
        base[tid] += add;
        __syncthreads();
    }
}

// ------------------------------------------------------------ partition

__global__ void k_valid_flags(const uint8_t* __restrict__ valid, uint32_t n, uint32_t* __restrict__ flags) {
    uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) flags[r] = bit_valid(valid, r) ? 1u : 0u;
}

__global__ void k_multi_valid_flags(const ColDev* __restrict__ cols, const uint32_t* __restrict__ attrs,
                                    uint32_t n_attrs, uint32_t n, uint32_t* __restrict__ flags) {
    uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    uint32_t f = 1;
    for (uint32_t a = 0; a < n_attrs; ++a) f &= bit_valid(cols[attrs[a]].valid, r) ? 1u : 0u;
    flags[r] = f;
}

// One thread per tile: binary search of the tile prefix for its block.
__global__ void k_tile_blocks(const uint64_t* __restrict__ tp, uint32_t n_blocks, uint64_t n_tiles,
                              uint32_t* __restrict__ tile_blk) {
    for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < n_tiles;
         t += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t lo = 0, hi = n_blocks - 1;
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) >> 1;
            if (tp[mid] <= t) lo = mid; else hi = mid - 1;
        }
        tile_blk[t] = lo;
    }
}

__global__ void k_size_flags(const uint32_t* __restrict__ size, uint32_t n, uint32_t min,
                             uint32_t* __restrict__ flags) {
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < n) flags[b] = size[b] >= min ? 1u : 0u;
}

__global__ void k_compact_rows(const uint32_t* __restrict__ flags, const uint32_t* __restrict__ dest,
                               uint32_t n, uint32_t* __restrict__ rows) {
    uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n && flags[r]) rows[dest[r]] = r;
}

__global__ void k_key_extract(const int64_t* __restrict__ vals, const uint8_t* __restrict__ valid, uint32_t n,
                              unsigned long long key_min, uint64_t* __restrict__ keys,
                              uint32_t* __restrict__ rows, const uint32_t* __restrict__ dest) {
    uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n || !bit_valid(valid, r)) return;
    uint32_t o = dest[r];
    keys[o] = order_key(vals[r]) - key_min;
    rows[o] = r;
}

__global__ void k_gather_key(const ColDev* __restrict__ cols, uint32_t attr, unsigned long long key_min,
                             const uint32_t* __restrict__ rows, uint32_t n, uint64_t* __restrict__ keys) {
    uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x < n) keys[x] = order_key(cols[attr].values[rows[x]]) - key_min;
}

__global__ void k_group_heads(const ColDev* __restrict__ cols, const uint32_t* __restrict__ attrs,
                              uint32_t n_attrs, const uint32_t* __restrict__ rows, uint32_t n,
                              uint32_t* __restrict__ head) {
    uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    uint32_t h = 1;
    if (x > 0) {
        uint32_t a = rows[x], b = rows[x - 1];
        h = 0;
        for (uint32_t k = 0; k < n_attrs; ++k) {
            const int64_t* v = cols[attrs[k]].values;
            if (v[a] != v[b]) h = 1;
        }
    }
    head[x] = h;
}

__global__ void k_group_start(const uint32_t* __restrict__ head, const uint32_t* __restrict__ gid,
                              uint32_t n, uint32_t* __restrict__ start) {
    uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x < n && head[x]) start[gid[x]] = x;
}

__device__ inline uint32_t group_size(const uint32_t* gstart, uint32_t g, uint32_t n_groups, uint32_t n_rows) {
    uint32_t e = (g + 1 < n_groups) ? gstart[g + 1] : n_rows;
    return e - gstart[g];
}

__global__ void k_ge2_flags(const uint32_t* __restrict__ gstart, uint32_t n_groups, uint32_t n_rows,
                            uint32_t* __restrict__ flags) {
    uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < n_groups) flags[g] = group_size(gstart, g, n_groups, n_rows) >= 2 ? 1u : 0u;
}

__global__ void k_block_table(const uint32_t* __restrict__ gstart, uint32_t n_groups, uint32_t n_rows,
                              const uint32_t* __restrict__ dest, uint32_t* __restrict__ blk_start,
                              uint32_t* __restrict__ blk_size, uint64_t* __restrict__ tiles,
                              unsigned long long* __restrict__ pairs) {
    uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long p = 0;
    if (g < n_groups) {
        uint32_t sz = group_size(gstart, g, n_groups, n_rows);
        if (sz >= 2) {
            uint32_t b = dest[g];
            blk_start[b] = gstart[g];
            blk_size[b] = sz;
            uint64_t T = (sz + kTile - 1) / kTile;
            tiles[b] = T * (T + 1) / 2;
            p = (unsigned long long)sz * (sz - 1) / 2;
        }
    }
    for (int o = 32; o > 0; o >>= 1) p += __shfl_xor(p, o);
    if ((threadIdx.x & 63) == 0 && p) atomicAdd(pairs, p);
}

__global__ void k_group_pairs(const uint32_t* __restrict__ gstart, uint32_t n_groups, uint32_t n_rows,
                              unsigned long long* __restrict__ pairs) {
    uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long p = 0;
    if (g < n_groups) {
        unsigned long long sz = group_size(gstart, g, n_groups, n_rows);
        p = sz * (sz - 1) / 2;
    }
    for (int o = 32; o > 0; o >>= 1) p += __shfl_xor(p, o);
    if ((threadIdx.x & 63) == 0 && p) atomicAdd(pairs, p);
}

// ------------------------------------------------------------ q-gram index

__device__ inline uint32_t str_len(const ColDev& c, uint32_t r) { return (uint32_t)(c.off[r + 1] - c.off[r]); }

// slots[r]: room reserved for row r's list (windows, or 1 for a short string)
__global__ void k_gram_slots(const ColDev* __restrict__ colp, uint32_t n, uint32_t q, uint64_t* __restrict__ slots) {
    uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const ColDev c = *colp;
    uint64_t s = 0;
    if (bit_valid(c.valid, r)) {
        uint32_t L = str_len(c, r);
        s = (L == 0) ? 0 : (L < q ? 1 : L - q + 1);
    }
    slots[r] = s;
}

// The signature bit of a q-gram code: bit (mix64(code) mod 64 W) of the
// row's W-word signature.
__device__ __forceinline__ uint32_t sig_bit(uint32_t code, uint32_t bits) { return (uint32_t)(mix64(code) & bits); }

// Rows of at most N windows (N a power of two <= 64): one thread per row
// holds its window codes in registers, padded with the largest code, sorts
// them with a bitonic network whose indices are all compile-time (so the
// keys never leave registers), and writes the distinct codes and the
// row's one-word signature (a bit per distinct code).  The pad value can
// equal a real q = 4 code; the first nw sorted keys are still the row's
// multiset because no pad is smaller than a real code.
template <int N>
__global__ __launch_bounds__(256) void k_gram_build_reg(const ColDev* __restrict__ colp, uint32_t n, uint32_t q,
                                                        const uint64_t* __restrict__ off,
                                                        uint32_t* __restrict__ codes, uint32_t* __restrict__ cnt,
                                                        uint8_t* __restrict__ flags, uint64_t* __restrict__ sig) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t out_cnt = 0;
    uint64_t m = 0;
    if (r < n) {
        const ColDev c = *colp;
        uint8_t f = 0;
        if (bit_valid(c.valid, r)) {
            const uint8_t* s = c.bytes + c.off[r];
            const uint32_t L = str_len(c, r);
            uint32_t* dst = codes + off[r];
            if (L > 0 && L < q) {
                uint32_t v = 0;
                for (uint32_t x = 0; x < L; ++x) v = (v << 8) | s[x];
                dst[0] = (L << 24) | v;
                m = 1ull << sig_bit((L << 24) | v, 63u);
                out_cnt = 1;
                f = 1;
            } else if (L >= q) {
                const uint32_t nw = L - q + 1;   // <= N (the launch checks the longest row)
                const uint32_t mask = (q == 4) ? 0xFFFFFFFFu : ((1u << (8 * q)) - 1u);
                // the string's bytes through aligned dword loads (one per
                // four bytes; the column's buffer is 16-byte aligned and has
                // 16 bytes of slack at its end), realigned with funnel shifts
                constexpr int kD = (N + 3 + 3) / 4 + 1;
                const uintptr_t addr = (uintptr_t)s;
                const uint32_t* wp = (const uint32_t*)(addr & ~(uintptr_t)3);
                const uint32_t sh = (uint32_t)(addr & 3);
                const uint32_t nd = (sh + L + 3) >> 2;   // dwords holding [s, s + L)
                uint32_t d[kD];
#pragma unroll
                for (int i = 0; i < kD; ++i) d[i] = (uint32_t)i < nd ? wp[i] : 0u;
                uint32_t b[N + 3];
#pragma unroll
                for (int i = 0; i + 1 < kD; ++i) {
                    const uint32_t a = __builtin_amdgcn_alignbyte(d[i + 1], d[i], sh);
#pragma unroll
                    for (int y = 0; y < 4; ++y)
                        if (4 * i + y < N + 3) b[4 * i + y] = (uint32_t)(4 * i + y) < L ? (a >> (8 * y)) & 0xFFu : 0u;
                }
                uint32_t k[N];
                uint32_t v = 0;   // the first q - 1 bytes (constant indices keep b in registers)
                if (q >= 2) v = b[0];
                if (q >= 3) v = (v << 8) | b[1];
                if (q >= 4) v = (v << 8) | b[2];
#pragma unroll
                for (int w = 0; w < N; ++w) {
                    // window w ends at byte w + q - 1 (q <= 4)
                    const uint32_t e = q == 1 ? b[w] : q == 2 ? b[w + 1] : q == 3 ? b[w + 2] : b[w + 3];
                    v = ((v << 8) | e) & mask;
                    k[w] = (uint32_t)w < nw ? v : 0xFFFFFFFFu;
                }
#pragma unroll
                for (int kk = 2; kk <= N; kk <<= 1) {
#pragma unroll
                    for (int j = kk >> 1; j > 0; j >>= 1) {
#pragma unroll
                        for (int i = 0; i < N; ++i) {
                            const int l = i ^ j;
                            if (l > i) {
                                const uint32_t a = k[i], bb = k[l];
                                const uint32_t lo = a < bb ? a : bb, hi = a < bb ? bb : a;
                                if ((i & kk) == 0) { k[i] = lo; k[l] = hi; }
                                else { k[i] = hi; k[l] = lo; }
                            }
                        }
                    }
                }
                uint32_t u = 0;
#pragma unroll
                for (int w = 0; w < N; ++w) {
                    if ((uint32_t)w < nw && (w == 0 || k[w] != k[w - 1])) {
                        dst[u] = k[w];
                        m |= 1ull << sig_bit(k[w], 63u);
                        ++u;
                    }
                }
                out_cnt = u;
            }
        }
        cnt[r] = out_cnt;
        flags[r] = f;
        sig[r] = m;
    }
}

__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Long rows: one wave per row.  The row's window codes go to the wave's LDS
// buffer of `cap` words (a power of two >= the longest row's window count),
// padded with the largest code, are bitonic-sorted by the 64 lanes, and
// the distinct values are compacted out with a ballot per 64 entries; each
// lane sets the signature bits of the codes it kept (kLongSigWords words)
// and the wave ORs them together.
__global__ __launch_bounds__(256) void k_gram_build_wave(const ColDev* __restrict__ colp, uint32_t n, uint32_t q,
                                                         const uint64_t* __restrict__ off,
                                                         uint32_t* __restrict__ codes, uint32_t* __restrict__ cnt,
                                                         uint8_t* __restrict__ flags, uint32_t cap,
                                                         uint64_t* __restrict__ sig) {
    extern __shared__ uint32_t gram_lds[];
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t* buf = gram_lds + (size_t)wave * cap;
    const ColDev c = *colp;
    const uint32_t mask = (q == 4) ? 0xFFFFFFFFu : ((1u << (8 * q)) - 1u);
    constexpr uint32_t kBits = 64u * kLongSigWords - 1u;
    for (uint32_t r = blockIdx.x * 4 + wave; r < n; r += gridDim.x * 4) {
        uint32_t out_cnt = 0;
        uint8_t f = 0;
        uint64_t m[kLongSigWords] = {0, 0, 0, 0};
        if (bit_valid(c.valid, r)) {
            const uint8_t* sp = c.bytes + c.off[r];
            const uint32_t L = str_len(c, r);
            uint32_t* dst = codes + off[r];
            if (L > 0 && L < q) {
                if (lane == 0) {
                    uint32_t v = 0;
                    for (uint32_t x = 0; x < L; ++x) v = (v << 8) | sp[x];
                    dst[0] = (L << 24) | v;
                    const uint32_t b = sig_bit((L << 24) | v, kBits);
#pragma unroll
                    for (uint32_t w = 0; w < kLongSigWords; ++w) m[w] |= (b >> 6) == w ? 1ull << (b & 63) : 0ull;
                }
                out_cnt = 1;
                f = 1;
            } else if (L >= q) {
                const uint32_t nw = L - q + 1;
                uint32_t P = 64;
                while (P < nw) P <<= 1;
                for (uint32_t w = lane; w < P; w += 64) {
                    uint32_t v = 0xFFFFFFFFu;
                    if (w < nw) {
                        v = 0;
                        for (uint32_t x = 0; x < q; ++x) v = (v << 8) | sp[w + x];
                        v &= mask;
                    }
                    buf[w] = v;
                }
                wave_lds_sync();
                for (uint32_t k = 2; k <= P; k <<= 1)
                    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                        for (uint32_t i = lane; i < P; i += 64) {
                            const uint32_t pj = i ^ j;
                            if (pj > i) {
                                const uint32_t a = buf[i], b = buf[pj];
                                const bool up = (i & k) == 0;
                                if (up ? a > b : a < b) {
                                    buf[i] = b;
                                    buf[pj] = a;
                                }
                            }
                        }
                        wave_lds_sync();
                    }
                for (uint32_t base = 0; base < nw; base += 64) {
                    const uint32_t i = base + lane;
                    const uint32_t x = i < nw ? buf[i] : 0u;
                    const bool keep = i < nw && (i == 0 || buf[i - 1] != x);
                    const uint64_t b = __ballot(keep);
                    const uint32_t rank = (uint32_t)__popcll(b & ((1ull << lane) - 1ull));
                    if (keep) {
                        dst[out_cnt + rank] = x;
                        const uint32_t sb = sig_bit(x, kBits);
#pragma unroll
                        for (uint32_t w = 0; w < kLongSigWords; ++w) m[w] |= (sb >> 6) == w ? 1ull << (sb & 63) : 0ull;
                    }
                    out_cnt += (uint32_t)__popcll(b);
                }
                wave_lds_sync();   // the buffer is reused by the next row
            }
        }
        // the wave's signature: OR over the lanes
#pragma unroll
        for (uint32_t w = 0; w < kLongSigWords; ++w)
            for (int o = 32; o > 0; o >>= 1) m[w] |= __shfl_xor(m[w], o);
        if (lane == 0) {
            cnt[r] = out_cnt;
            flags[r] = f;
        }
        if (lane < kLongSigWords) {
            uint64_t v = m[0];
#pragma unroll
            for (uint32_t w = 1; w < kLongSigWords; ++w) v = lane == w ? m[w] : v;
            sig[(size_t)r * kLongSigWords + lane] = v;
        }
    }
}

// ------------------------------------------------------------ features

// bit (c mod 64) for every byte c of the string: a substitution changes at
// most one set bit on each side, an insertion or deletion at most one, so
// the edit distance is at least max(|sig_a \ sig_b|, |sig_b \ sig_a|)
__global__ void k_char_sig(const ColDev* __restrict__ colp, uint32_t n, uint64_t* __restrict__ sig) {
    uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const ColDev c = *colp;
    uint64_t m = 0;
    if (bit_valid(c.valid, r)) {
        const uint8_t* s = c.bytes + c.off[r];
        const uint32_t L = str_len(c, r);
        for (uint32_t x = 0; x < L; x += 8) {   // eight independent loads per batch
            uint32_t v[8];
#pragma unroll
            for (uint32_t k = 0; k < 8; ++k) v[k] = x + k < L ? s[x + k] : 0u;
#pragma unroll
            for (uint32_t k = 0; k < 8; ++k)
                if (x + k < L) m |= 1ull << (v[k] & 63);
        }
    }
    sig[r] = m;
}

// bit (hash(code) mod 64 W) of a W-word signature for every distinct q-gram
// code of the row: a gram in A whose bit is absent from sig_B is not in B,
// so |A & B| <= |A| - |sig_A \ sig_B|
__global__ void k_gather_features(const GatherParams P) {
    const uint64_t p = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (p >= P.stride) return;
    const uint64_t n = P.stride;
    const uint32_t y = blockIdx.y;
    const bool pad = p >= P.n;
    const uint32_t row = pad ? 0u : P.perm[p];
    if (y == 0) {   // row id and validity mask
        uint32_t vmask = 0;
        if (!pad) {
            for (uint32_t x = 0; x < P.n_int; ++x) vmask |= (bit_valid(P.int_valid[x], row) ? 1u : 0u) << x;
            for (uint32_t x = 0; x < P.n_str; ++x) vmask |= (bit_valid(P.str_valid[x], row) ? 1u : 0u) << (16 + x);
            for (uint32_t x = 0; x < P.n_gram; ++x) vmask |= (bit_valid(P.gram_valid[x], row) ? 1u : 0u) << (24 + x);
        }
        P.f32[p] = pad ? 0u : row;
        P.f32[n + p] = vmask;
        return;
    }
    uint32_t x = y - 1;
    if (x < P.n_int) {
        const bool v = !pad && bit_valid(P.int_valid[x], row);
        P.f64[x * n + p] = v ? (uint64_t)P.int_vals[x][row] : 0ull;
        return;
    }
    x -= P.n_int;
    if (x < P.n_str) {
        const bool v = !pad && bit_valid(P.str_valid[x], row);
        P.f64[(P.n_int + x) * n + p] = v ? P.csig[x][row] : 0ull;
        P.f32[(2 + x) * n + p] = v ? (uint32_t)(P.str_off[x][row + 1] - P.str_off[x][row]) : 0u;
        return;
    }
    x -= P.n_str;
    const bool v = !pad && bit_valid(P.gram_valid[x], row);
    const uint32_t W = P.gram_words[x];
    uint32_t pop = 0;
    for (uint32_t w = 0; w < W; ++w) {
        const uint64_t sig = v ? P.gsig[x][(size_t)row * W + w] : 0ull;
        P.f64[(P.n_int + P.n_str + P.gram_col[x] + w) * n + p] = sig;
        pop += (uint32_t)__popcll(sig);
    }
    const uint32_t cnt = v ? P.gram_cnt[x][row] : 0u;
    P.f32[(2 + P.n_str + x) * n + p] = v ? (cnt | ((uint32_t)(P.gram_flags[x][row] & 1) << 31)) : 0u;
    // the Jaccard-filter word: 1 marks a missing value (pads: 0)
    P.f32[(2 + P.n_str + P.n_gram + x) * n + p] =
        v ? ((cnt - pop) << 16) | cnt : pad ? 0u : 1u;
}

// ------------------------------------------------------------ LSH histogram

__device__ inline uint64_t fnv1a64(const uint8_t* s, uint32_t L) {
    uint64_t h = 0xCBF29CE484222325ull;
    for (uint32_t x = 0; x < L; ++x) { h ^= s[x]; h *= 0x100000001B3ull; }
    return h;
}

// minimum over the q-gram set of mix64((len << 32) | big-endian bytes)
__device__ inline uint64_t minhash(const uint8_t* s, uint32_t L, uint32_t q) {
    if (L == 0) return 0;
    if (L < q) {
        uint64_t v = 0;
        for (uint32_t x = 0; x < L; ++x) v = (v << 8) | s[x];
        return mix64(((uint64_t)L << 32) | v);
    }
    uint64_t best = ~0ull;
    const uint64_t mask = (1ull << (8 * q)) - 1ull;
    uint64_t v = 0;
    for (uint32_t x = 0; x + 1 < q; ++x) v = (v << 8) | s[x];
    // the string's bytes in batches of four independent loads
    uint32_t ch[4];
    for (uint32_t w = 0; w + q <= L; ++w) {
        if ((w & 3) == 0) {
#pragma unroll
            for (uint32_t k = 0; k < 4; ++k) ch[k] = w + q - 1 + k < L ? s[w + q - 1 + k] : 0u;
        }
        v = ((v << 8) | ch[w & 3]) & mask;
        uint64_t h = mix64(((uint64_t)q << 32) | v);
        best = h < best ? h : best;
    }
    return best;
}

__device__ inline int64_t floor_div(int64_t v, int64_t d) {
    // floor(v / (d + 1)) for d >= 0
    if (d == INT64_MAX) return v < 0 ? -1 : 0;
    int64_t w = d + 1;
    int64_t qq = v / w, rr = v % w;
    if (rr != 0 && v < 0) qq -= 1;
    return qq;
}

// op: 0 EQ, 1 ED (2-gram MinHash), 2 JACCARD (q-gram MinHash), 3 ABSDIFF
__global__ void k_lsh_hist(const ColDev* __restrict__ colp, uint32_t n, int op, uint32_t q, int64_t d,
                           unsigned long long* __restrict__ hist) {
    __shared__ unsigned int h[kLshK];
    for (int x = threadIdx.x; x < kLshK; x += blockDim.x) h[x] = 0;
    __syncthreads();
    const ColDev c = *colp;
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        if (!bit_valid(c.valid, r)) continue;
        uint64_t hv;
        if (c.type == COL_STRING) {
            const uint8_t* s = c.bytes + c.off[r];
            uint32_t L = str_len(c, r);
            if (op == 0) hv = mix64(fnv1a64(s, L));
            else if (op == 1) hv = minhash(s, L, 2);
            else hv = minhash(s, L, q);
        } else {
            int64_t v = c.values[r];
            if (op == 3) v = floor_div(v, d);
            hv = mix64((uint64_t)v);
        }
        atomicAdd(&h[hv % kLshK], 1u);
    }
    __syncthreads();
    for (int x = threadIdx.x; x < kLshK; x += blockDim.x)
        if (h[x]) atomicAdd(&hist[x], (unsigned long long)h[x]);
}

__global__ void k_copy_u64(const uint64_t* __restrict__ in, uint64_t* __restrict__ out, uint64_t n) {
    for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < n; x += (uint64_t)gridDim.x * blockDim.x)
        out[x] = in[x];
}

inline unsigned grid_for(uint64_t n, unsigned cap = 65535u * 4) {
    uint64_t g = (n + kBlock - 1) / kBlock;
    if (g == 0) g = 1;
    return (unsigned)(g < cap ? g : cap);
}

}  // namespace

hipError_t launch_string_stats(const uint64_t* off, uint32_t n, uint32_t* d_max_len,
                               unsigned long long* d_total, uint32_t* d_bad, hipStream_t s) {
    k_string_stats<<<grid_for(n, 512), kBlock, 0, s>>>(off, n, d_max_len, d_total, d_bad);
    return hipGetLastError();
}

hipError_t launch_minmax_u64(const int64_t* vals, const uint8_t* valid, uint32_t n,
                             unsigned long long* d_min, unsigned long long* d_max,
                             unsigned int* d_nvalid, hipStream_t s) {
    k_minmax<<<grid_for(n, 512), kBlock, 0, s>>>(vals, valid, n, d_min, d_max, d_nvalid);
    return hipGetLastError();
}

size_t scan_tmp_elems(size_t n) {
    size_t total = 0;
    size_t m = n;
    while (m > kScanChunk) {
        m = (m + kScanChunk - 1) / kScanChunk;
        total += m;
    }
    return total + 1;
}

hipError_t launch_exclusive_scan_u32(const uint32_t* in, uint32_t* out, size_t n, uint32_t* tmp,
                                     hipStream_t s) {
    return scan_impl<uint32_t>(in, out, n, tmp, s);
}

hipError_t launch_exclusive_scan_u64(const uint64_t* in, uint64_t* out, size_t n, uint64_t* tmp,
                                     hipStream_t s) {
    return scan_impl<uint64_t>(in, out, n, tmp, s);
}

size_t radix_tmp_bytes(uint32_t n) {
    size_t G = (n + kRsChunk - 1) / kRsChunk;
    if (G == 0) G = 1;
    size_t hist = 256 * G;
    return (hist * 2 + scan_tmp_elems(hist)) * sizeof(uint32_t);
}

hipError_t radix_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt,
                            uint32_t n, const int* shifts, int n_shifts, void* tmp,
                            bool* result_in_alt, hipStream_t s) {
    *result_in_alt = false;
    if (n <= 1) return hipSuccess;
    uint32_t G = (n + kRsChunk - 1) / kRsChunk;
    size_t H = (size_t)256 * G;
    uint32_t* hist = (uint32_t*)tmp;
    uint32_t* offs = hist + H;
    uint32_t* stmp = offs + H;
    uint64_t* kin = keys; uint32_t* vin = vals;
    uint64_t* kout = keys_alt; uint32_t* vout = vals_alt;
    for (int p = 0; p < n_shifts; ++p) {
        k_rs_hist<<<G, kBlock, 0, s>>>(kin, n, shifts[p], hist, G);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = scan_impl<uint32_t>(hist, offs, H, stmp, s);
        if (e != hipSuccess) return e;
        k_rs_scatter<<<G, kBlock, 0, s>>>(kin, vin, kout, vout, n, shifts[p], offs, G);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        uint64_t* tk = kin; kin = kout; kout = tk;
        uint32_t* tv = vin; vin = vout; vout = tv;
        *result_in_alt = !*result_in_alt;
    }
    return hipSuccess;
}

hipError_t launch_valid_flags(const uint8_t* valid, uint32_t n, uint32_t* flags, hipStream_t s) {
    k_valid_flags<<<grid_for(n, 1u << 30), kBlock, 0, s>>>(valid, n, flags);
    return hipGetLastError();
}

hipError_t launch_multi_valid_flags(const ColDev* cols, const uint32_t* attrs, uint32_t n_attrs,
                                    uint32_t n, uint32_t* flags, hipStream_t s) {
    k_multi_valid_flags<<<grid_for(n, 1u << 30), kBlock, 0, s>>>(cols, attrs, n_attrs, n, flags);
    return hipGetLastError();
}

hipError_t launch_compact_rows(const uint32_t* flags, const uint32_t* dest, uint32_t n,
                               uint32_t* rows, hipStream_t s) {
    k_compact_rows<<<grid_for(n, 1u << 30), kBlock, 0, s>>>(flags, dest, n, rows);
    return hipGetLastError();
}

hipError_t launch_tile_blocks(const uint64_t* tile_prefix, uint32_t n_blocks, uint64_t n_tiles, uint32_t* tile_blk,
                              hipStream_t s) {
    if (n_tiles == 0 || n_blocks == 0) return hipSuccess;
    k_tile_blocks<<<grid_for(n_tiles, 1u << 16), kBlock, 0, s>>>(tile_prefix, n_blocks, n_tiles, tile_blk);
    return hipGetLastError();
}

hipError_t launch_size_flags(const uint32_t* size, uint32_t n, uint32_t min, uint32_t* flags, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_size_flags<<<grid_for(n, 1u << 30), kBlock, 0, s>>>(size, n, min, flags);
    return hipGetLastError();
}

hipError_t launch_key_extract(const int64_t* vals, const uint8_t* valid, uint32_t n,
                              unsigned long long key_min, uint64_t* keys, uint32_t* rows,
                              const uint32_t* dest, hipStream_t s) {
    k_key_extract<<<grid_for(n, 1u << 30), kBlock, 0, s>>>(vals, valid, n, key_min, keys, rows, dest);
    return hipGetLastError();
}

hipError_t launch_gather_key(const ColDev* cols, uint32_t attr, unsigned long long key_min,
                             const uint32_t* rows, uint32_t n, uint64_t* keys, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_gather_key<<<grid_for(n, 1u << 30), kBlock, 0, s>>>(cols, attr, key_min, rows, n, keys);
    return hipGetLastError();
}

hipError_t launch_group_heads(const ColDev* cols, const uint32_t* attrs, uint32_t n_attrs,
                              const uint32_t* rows, uint32_t n, uint32_t* head, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_group_heads<<<grid_for(n, 1u << 30), kBlock, 0, s>>>(cols, attrs, n_attrs, rows, n, head);
    return hipGetLastError();
}

hipError_t launch_group_sizes(const uint32_t* head, const uint32_t* gid, uint32_t n,
                              uint32_t n_groups, uint32_t* start, hipStream_t s) {
    (void)n_groups;
    if (n == 0) return hipSuccess;
    k_group_start<<<grid_for(n, 1u << 30), kBlock, 0, s>>>(head, gid, n, start);
    return hipGetLastError();
}

hipError_t launch_ge2_flags(const uint32_t* gstart, uint32_t n_groups, uint32_t n_rows,
                            uint32_t* flags, hipStream_t s) {
    if (n_groups == 0) return hipSuccess;
    k_ge2_flags<<<grid_for(n_groups, 1u << 30), kBlock, 0, s>>>(gstart, n_groups, n_rows, flags);
    return hipGetLastError();
}

hipError_t launch_block_table(const uint32_t* gstart, uint32_t n_groups, uint32_t n_rows,
                              const uint32_t* dest, uint32_t* blk_start, uint32_t* blk_size,
                              uint64_t* tiles, unsigned long long* pairs, hipStream_t s) {
    if (n_groups == 0) return hipSuccess;
    k_block_table<<<grid_for(n_groups, 1u << 30), kBlock, 0, s>>>(gstart, n_groups, n_rows, dest,
                                                                  blk_start, blk_size, tiles, pairs);
    return hipGetLastError();
}

hipError_t launch_group_pairs(const uint32_t* gstart, uint32_t n_groups, uint32_t n_rows,
                              unsigned long long* pairs, hipStream_t s) {
    if (n_groups == 0) return hipSuccess;
    k_group_pairs<<<grid_for(n_groups, 1u << 30), kBlock, 0, s>>>(gstart, n_groups, n_rows, pairs);
    return hipGetLastError();
}

hipError_t launch_gram_slots(const ColDev* col, uint32_t n, uint32_t q, uint64_t* slots, hipStream_t s) {
    k_gram_slots<<<grid_for(n, 1u << 30), kBlock, 0, s>>>(col, n, q, slots);
    return hipGetLastError();
}

hipError_t launch_gram_build(const ColDev* col, uint32_t n, uint32_t q, const uint64_t* off,
                             uint32_t* codes, uint32_t* cnt, uint8_t* flags, uint64_t* sig, uint32_t max_windows,
                             hipStream_t s) {
    if (max_windows > 4096) return hipErrorInvalidValue;   // Jaccard attributes hold <= 4096-byte strings
    if (max_windows > 64) {
        // long rows: a wave per row, sorting in a power-of-two LDS buffer
        uint32_t cap = 64;
        while (cap < max_windows) cap <<= 1;
        const size_t lds = (size_t)4 * cap * 4;
        if (lds > 64 * 1024) {
            hipError_t e = hipFuncSetAttribute((const void*)k_gram_build_wave,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>((n + 3) / 4, 65536));
        k_gram_build_wave<<<grid, 256, lds, s>>>(col, n, q, off, codes, cnt, flags, cap, sig);
        return hipGetLastError();
    }
    // short rows: a thread per row, sorting in registers
    const uint32_t grid = std::max<uint32_t>(1, (n + 255) / 256);
    if (max_windows <= 8)
        k_gram_build_reg<8><<<grid, 256, 0, s>>>(col, n, q, off, codes, cnt, flags, sig);
    else if (max_windows <= 16)
        k_gram_build_reg<16><<<grid, 256, 0, s>>>(col, n, q, off, codes, cnt, flags, sig);
    else if (max_windows <= 32)
        k_gram_build_reg<32><<<grid, 256, 0, s>>>(col, n, q, off, codes, cnt, flags, sig);
    else
        k_gram_build_reg<64><<<grid, 256, 0, s>>>(col, n, q, off, codes, cnt, flags, sig);
    return hipGetLastError();
}


hipError_t launch_char_sig(const ColDev* col, uint32_t n, uint64_t* sig, hipStream_t s) {
    k_char_sig<<<grid_for(n, 1u << 30), kBlock, 0, s>>>(col, n, sig);
    return hipGetLastError();
}


// One wave per 64 rows: each lane builds its row's record (the features
// the column-wise gather would write at the row's position) in LDS, at an
// odd word stride so the lanes' rows fall in distinct banks; the wave then
// writes the 64 records out as one contiguous run of full cache lines.
__global__ __launch_bounds__(64) void k_pack_records(const GatherParams P) {
    extern __shared__ uint32_t rec_lds[];
    const uint32_t lane = threadIdx.x, row0 = blockIdx.x * 64u, row = row0 + lane;
    const uint32_t RW = P.rec_words, RWp = RW + 1;
    uint32_t* rec = rec_lds + lane * RWp;
    if (row < P.n_rows) {
        uint32_t vmask = 0;
        for (uint32_t x = 0; x < P.n_int; ++x) vmask |= (bit_valid(P.int_valid[x], row) ? 1u : 0u) << x;
        for (uint32_t x = 0; x < P.n_str; ++x) vmask |= (bit_valid(P.str_valid[x], row) ? 1u : 0u) << (16 + x);
        for (uint32_t x = 0; x < P.n_gram; ++x) vmask |= (bit_valid(P.gram_valid[x], row) ? 1u : 0u) << (24 + x);
        auto put64 = [&](uint32_t col, uint64_t v) {
            rec[2 * col] = (uint32_t)v;
            rec[2 * col + 1] = (uint32_t)(v >> 32);
        };
        uint32_t* r32 = rec + 2 * P.n64 - 1;   // f32 column k at r32[k], k >= 1
        r32[1] = vmask;
        for (uint32_t x = 0; x < P.n_int; ++x) {
            const bool v = (vmask >> x) & 1;
            put64(x, v ? (uint64_t)P.int_vals[x][row] : 0ull);
        }
        for (uint32_t x = 0; x < P.n_str; ++x) {
            const bool v = (vmask >> (16 + x)) & 1;
            put64(P.n_int + x, v ? P.csig[x][row] : 0ull);
            r32[2 + x] = v ? (uint32_t)(P.str_off[x][row + 1] - P.str_off[x][row]) : 0u;
        }
        for (uint32_t x = 0; x < P.n_gram; ++x) {
            const bool v = (vmask >> (24 + x)) & 1;
            const uint32_t W = P.gram_words[x];
            uint32_t pop = 0;
            for (uint32_t w = 0; w < W; ++w) {
                const uint64_t sig = v ? P.gsig[x][(size_t)row * W + w] : 0ull;
                put64(P.n_int + P.n_str + P.gram_col[x] + w, sig);
                pop += (uint32_t)__popcll(sig);
            }
            const uint32_t cnt = v ? P.gram_cnt[x][row] : 0u;
            r32[2 + P.n_str + x] = v ? (cnt | ((uint32_t)(P.gram_flags[x][row] & 1) << 31)) : 0u;
            // the Jaccard-filter word: 1 marks a missing value
            r32[2 + P.n_str + P.n_gram + x] = v ? ((cnt - pop) << 16) | cnt : 1u;
        }
        for (uint32_t w = 2 * P.n64 + P.n32 - 1; w < RW; ++w) rec[w] = 0u;
    }
    __syncthreads();
    const uint32_t rows_here = min(64u, P.n_rows - row0);
    uint32_t* dst = P.rec + (size_t)row0 * RW;
    for (uint32_t q = 0; q < rows_here; ++q)
        for (uint32_t w = lane; w < RW; w += 64) dst[(size_t)q * RW + w] = rec_lds[q * RWp + w];
}

// One wave per 64 positions: the wave reads the 64 permuted rows' records
// one record per step (a contiguous run, lane w taking word w) into LDS;
// each lane then splits its position's record into the feature columns
// (pads: zeros, row id 0), one coalesced store per column.
__global__ __launch_bounds__(64) void k_gather_records(const GatherParams P) {
    extern __shared__ uint32_t rec_lds[];
    const uint32_t lane = threadIdx.x;
    const uint64_t p0 = (uint64_t)blockIdx.x * 64u, p = p0 + lane;
    const uint64_t n = P.stride;
    const uint32_t RW = P.rec_words, RWp = RW + 1;
    const bool pad = p >= P.n;
    const uint32_t row = pad ? 0u : P.perm[p];
    for (uint32_t q = 0; q < 64; ++q) {
        const uint32_t rq = __builtin_amdgcn_readlane(row, q);
        const bool padq = p0 + q >= P.n;
        const uint32_t* src = P.rec + (size_t)rq * RW;
        for (uint32_t w = lane; w < RW; w += 64) rec_lds[q * RWp + w] = padq ? 0u : src[w];
    }
    __syncthreads();
    if (p >= P.stride) return;
    const uint32_t* rec = rec_lds + lane * RWp;
    P.f32[p] = row;
    const uint32_t w64 = 2 * P.n64, wend = w64 + P.n32 - 1;
    for (uint32_t k = 0; 2 * k < w64; ++k) P.f64[(uint64_t)k * n + p] = ((uint64_t)rec[2 * k + 1] << 32) | rec[2 * k];
    for (uint32_t w = w64; w < wend; ++w) P.f32[(uint64_t)(1 + w - w64) * n + p] = rec[w];
}

hipError_t launch_pack_records(const GatherParams& p, hipStream_t s) {
    if (p.n_rows == 0) return hipSuccess;
    const size_t lds = (size_t)64 * (p.rec_words + 1) * 4;
    if (lds > 64 * 1024) return hipErrorInvalidValue;
    k_pack_records<<<(p.n_rows + 63) / 64, 64, lds, s>>>(p);
    return hipGetLastError();
}

hipError_t launch_gather_records(const GatherParams& p, hipStream_t s) {
    if (p.n == 0) return hipSuccess;
    const size_t lds = (size_t)64 * (p.rec_words + 1) * 4;
    if (lds > 64 * 1024) return hipErrorInvalidValue;
    k_gather_records<<<(unsigned)((p.stride + 63) / 64), 64, lds, s>>>(p);
    return hipGetLastError();
}

hipError_t launch_gather_features(const GatherParams& p, hipStream_t s) {
    if (p.n == 0) return hipSuccess;
    const dim3 grid(grid_for(p.stride, 1u << 30), 1 + p.n_int + p.n_str + p.n_gram);
    k_gather_features<<<grid, kBlock, 0, s>>>(p);
    return hipGetLastError();
}

hipError_t launch_lsh_hist(const ColDev* col, uint32_t n, int op, uint32_t q, int64_t d,
                           unsigned long long* hist, hipStream_t s) {
    k_lsh_hist<<<grid_for(n, 1024), kBlock, 0, s>>>(col, n, op, q, d, hist);
    return hipGetLastError();
}

hipError_t launch_copy_u64(const uint64_t* in, uint64_t* out, uint64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_copy_u64<<<grid_for(n, 4096), kBlock, 0, s>>>(in, out, n);
    return hipGetLastError();
}

}  // namespace hb
