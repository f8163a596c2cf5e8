/*
 * hbgen — seeded synthetic relations for rule-based blocking.
 *
 * This file holds no part of the blocking method: it only draws tuples.
 * It stands in for the paper's real datasets (Section 6, Table 2), which
 * are not available; every input is a deterministic function of the seed.
 *
 * Random numbers: xoshiro256** (Blackman and Vigna, "Scrambled linear
 * pseudorandom number generators", 2021) seeded through splitmix64
 * (Steele, Lea and Flood, OOPSLA 2014).  Each attribute draws from its own
 * stream, seeded with splitmix64(seed ^ (attribute index + 1)).
 *
 * Attribute kinds:
 *   HBGEN_STRING  length U[min_len, max_len] over a fixed alphabet
 *   HBGEN_WORDS   words from a pseudo-word vocabulary with Zipf word
 *                 frequencies, cut to a length U[min_len, max_len]
 *   HBGEN_ZIPF    categorical key, value rank r drawn with P(r) ~ r^-s over
 *                 n_values ranks; a value held by more than `cap` base tuples
 *                 is split into ceil(count/cap) distinct codes ("capped Zipf")
 *   HBGEN_CODES   categorical key, uniform over n_values distinct random
 *                 codes in [lo, hi]
 *   HBGEN_INT     int64 uniform in [lo, hi]
 *   HBGEN_KEYED   string correlated with an earlier key attribute `dep`:
 *                 each key code v is "pinned" with probability dep_p (a
 *                 draw from a stream seeded by the code); base tuples with a
 *                 pinned code share one string drawn from that stream, the
 *                 others draw like HBGEN_STRING (a city column under a zip
 *                 code, say: constant in some blocks, free in others)
 *
 * Duplicates: each duplicate copies a uniformly drawn base tuple (keys are
 * inherited), then applies E ~ U[edit_min, edit_max] character edits, each
 * on a uniformly drawn editable string attribute, of a uniformly drawn type
 * (substitute / insert / delete) at a uniform position, the new character
 * drawn from that attribute's alphabet; each int attribute with
 * int_p > 0 is shifted by U{-int_d..int_d} with probability int_p.
 * The final row order is a seeded random permutation of base + duplicates.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define HBGEN_STRING 0
#define HBGEN_WORDS 1
#define HBGEN_ZIPF 2
#define HBGEN_CODES 3
#define HBGEN_INT 4
#define HBGEN_KEYED 5

typedef struct {
    int32_t kind;
    int32_t alphabet;      /* 0: a-z, 1: a-z 0-9 space, 2: a-z space */
    uint32_t min_len, max_len;
    int32_t editable;      /* 1: duplicates may edit this string attribute */
    double zipf_s;         /* ZIPF exponent (also the word-frequency exponent for WORDS) */
    uint32_t n_values;     /* ZIPF / CODES value count; WORDS vocabulary size */
    uint32_t cap;          /* ZIPF cap on base tuples per code (0 = none) */
    int64_t lo, hi;        /* INT / CODES range */
    double int_p;          /* INT duplicate perturbation probability */
    int64_t int_d;         /* INT duplicate perturbation magnitude */
    int32_t dep;           /* KEYED: index of the (earlier) key attribute */
    double dep_p;          /* KEYED: probability that a key code is pinned */
} hbgen_attr;

typedef struct {
    uint64_t seed;
    uint32_t n_base, n_dup;
    uint32_t edit_min, edit_max;
    uint32_t n_attrs;
} hbgen_spec;

/* Output buffers are allocated by the caller:
 *   strings: offsets[n+1] (u64) and bytes[capacity]; ints/keys: values[n] (i64)
 * dup_src[n]: -1 for a base tuple, else the row of its source tuple. */
typedef struct {
    uint64_t* offsets;
    uint8_t* bytes;
    uint64_t bytes_cap;
    int64_t* values;
} hbgen_out_attr;

static inline uint64_t sm64(uint64_t* x) {
    uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

typedef struct { uint64_t s[4]; } xo256;

static inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static void xo_seed(xo256* r, uint64_t seed) {
    uint64_t x = seed;
    for (int i = 0; i < 4; ++i) r->s[i] = sm64(&x);
}

static inline uint64_t xo_next(xo256* r) {
    uint64_t* s = r->s;
    uint64_t result = rotl(s[1] * 5, 7) * 9;
    uint64_t t = s[1] << 17;
    s[2] ^= s[0]; s[3] ^= s[1]; s[1] ^= s[2]; s[0] ^= s[3];
    s[2] ^= t; s[3] = rotl(s[3], 45);
    return result;
}

/* uniform integer in [0, n) by Lemire's multiply-shift with rejection */
static inline uint64_t xo_below(xo256* r, uint64_t n) {
    if (n <= 1) return 0;
    for (;;) {
        uint64_t x = xo_next(r);
        __uint128_t m = (__uint128_t)x * n;
        uint64_t lo = (uint64_t)m;
        if (lo >= n) return (uint64_t)(m >> 64);
        uint64_t thr = (0 - n) % n;
        if (lo >= thr) return (uint64_t)(m >> 64);
    }
}

static inline double xo_unit(xo256* r) { return (double)(xo_next(r) >> 11) * (1.0 / 9007199254740992.0); }

static const char* ALPHA[3] = {
    "abcdefghijklmnopqrstuvwxyz",
    "abcdefghijklmnopqrstuvwxyz0123456789 ",
    "abcdefghijklmnopqrstuvwxyz ",
};

static uint64_t attr_seed(uint64_t seed, uint32_t a) {
    uint64_t x = seed ^ (uint64_t)(a + 1);
    return sm64(&x);
}

/* cumulative Zipf weights over ranks 1..n, normalised to 1 */
static double* zipf_cdf(uint32_t n, double s) {
    double* c = (double*)malloc(sizeof(double) * n);
    double acc = 0.0;
    for (uint32_t r = 0; r < n; ++r) { acc += pow((double)(r + 1), -s); c[r] = acc; }
    for (uint32_t r = 0; r < n; ++r) c[r] /= acc;
    return c;
}

static uint32_t zipf_draw(xo256* r, const double* cdf, uint32_t n) {
    double u = xo_unit(r);
    uint32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        uint32_t mid = (lo + hi) / 2;
        if (cdf[mid] < u) lo = mid + 1; else hi = mid;
    }
    return lo;
}

/* Strings are built in per-row scratch (max length after edits is
 * max_len + edit_max, far below this bound), then packed. */
#define HBGEN_MAXSTR 4096

typedef struct {
    char** words; uint32_t* wlen; uint32_t n; double* cdf;
} vocab;

static void vocab_build(vocab* v, uint32_t n, double s, xo256* r) {
    v->n = n;
    v->words = (char**)malloc(sizeof(char*) * n);
    v->wlen = (uint32_t*)malloc(sizeof(uint32_t) * n);
    for (uint32_t w = 0; w < n; ++w) {
        uint32_t L = 2 + (uint32_t)xo_below(r, 9); /* 2..10 */
        v->words[w] = (char*)malloc(L);
        v->wlen[w] = L;
        for (uint32_t k = 0; k < L; ++k) v->words[w][k] = ALPHA[0][xo_below(r, 26)];
    }
    v->cdf = zipf_cdf(n, s);
}

static void vocab_free(vocab* v) {
    for (uint32_t w = 0; w < v->n; ++w) free(v->words[w]);
    free(v->words); free(v->wlen); free(v->cdf);
}

typedef struct { char* p; uint32_t len; } sbuf;

/* returns 0 on success, -1 if a string buffer would overflow, -2 on bad spec */
int hbgen_generate(const hbgen_spec* spec, const hbgen_attr* attrs,
                   hbgen_out_attr* out, int64_t* dup_src, uint64_t* bytes_used) {
    const uint32_t nb = spec->n_base, nd = spec->n_dup, n = nb + nd;
    const uint32_t na = spec->n_attrs;
    if (n == 0 || na == 0) return -2;
    for (uint32_t a = 0; a < na; ++a) {
        const hbgen_attr* at = &attrs[a];
        if (at->kind == HBGEN_STRING || at->kind == HBGEN_WORDS || at->kind == HBGEN_KEYED) {
            if (at->min_len > at->max_len || at->max_len + spec->edit_max >= HBGEN_MAXSTR) return -2;
            if (at->kind != HBGEN_WORDS && (at->alphabet < 0 || at->alphabet > 2)) return -2;
            if (at->kind == HBGEN_KEYED &&
                (at->dep < 0 || (uint32_t)at->dep >= a ||
                 (attrs[at->dep].kind != HBGEN_ZIPF && attrs[at->dep].kind != HBGEN_CODES)))
                return -2;
            if (at->kind == HBGEN_WORDS && at->n_values == 0) return -2;
        } else if (at->kind == HBGEN_ZIPF) {
            if (at->n_values == 0) return -2;
        } else if (at->kind == HBGEN_CODES) {
            if (at->n_values == 0 || at->hi < at->lo || (uint64_t)(at->hi - at->lo) + 1 < at->n_values) return -2;
        } else if (at->kind == HBGEN_INT) {
            if (at->hi < at->lo) return -2;
        } else {
            return -2;
        }
    }

    /* base tuples, in generation order: rows 0..nb-1 of a staging table */
    sbuf* sv = (sbuf*)calloc((size_t)n * na, sizeof(sbuf));
    int64_t* iv = (int64_t*)calloc((size_t)n * na, sizeof(int64_t));
    int64_t* src = (int64_t*)malloc(sizeof(int64_t) * n);
    char tmp[HBGEN_MAXSTR];
    int rc = 0;

    for (uint32_t a = 0; a < na; ++a) {
        const hbgen_attr* at = &attrs[a];
        xo256 r; xo_seed(&r, attr_seed(spec->seed, a));
        if (at->kind == HBGEN_STRING) {
            const char* al = ALPHA[at->alphabet];
            uint32_t asz = (uint32_t)strlen(al);
            for (uint32_t i = 0; i < nb; ++i) {
                uint32_t L = at->min_len + (uint32_t)xo_below(&r, (uint64_t)(at->max_len - at->min_len) + 1);
                char* p = (char*)malloc(L ? L : 1);
                for (uint32_t k = 0; k < L; ++k) p[k] = al[xo_below(&r, asz)];
                sv[(size_t)i * na + a].p = p; sv[(size_t)i * na + a].len = L;
            }
        } else if (at->kind == HBGEN_KEYED) {
            const char* al = ALPHA[at->alphabet];
            uint32_t asz = (uint32_t)strlen(al);
            const uint64_t span = (uint64_t)(at->max_len - at->min_len) + 1;
            for (uint32_t i = 0; i < nb; ++i) {
                const int64_t v = iv[(size_t)i * na + at->dep];
                xo256 rv; xo_seed(&rv, attr_seed(spec->seed ^ ((uint64_t)v * 0x9E3779B97F4A7C15ull), a + 0x100u));
                xo256* src_r = xo_unit(&rv) < at->dep_p ? &rv : &r;
                uint32_t L = at->min_len + (uint32_t)xo_below(src_r, span);
                char* p = (char*)malloc(L ? L : 1);
                for (uint32_t k = 0; k < L; ++k) p[k] = al[xo_below(src_r, asz)];
                sv[(size_t)i * na + a].p = p; sv[(size_t)i * na + a].len = L;
            }
        } else if (at->kind == HBGEN_WORDS) {
            vocab v; vocab_build(&v, at->n_values, at->zipf_s, &r);
            for (uint32_t i = 0; i < nb; ++i) {
                uint32_t L = at->min_len + (uint32_t)xo_below(&r, (uint64_t)(at->max_len - at->min_len) + 1);
                uint32_t len = 0;
                while (len < L) {
                    uint32_t w = zipf_draw(&r, v.cdf, v.n);
                    if (len > 0) tmp[len++] = ' ';
                    for (uint32_t k = 0; k < v.wlen[w] && len < L; ++k) tmp[len++] = v.words[w][k];
                }
                if (len > L) len = L;
                char* p = (char*)malloc(len ? len : 1);
                memcpy(p, tmp, len);
                sv[(size_t)i * na + a].p = p; sv[(size_t)i * na + a].len = len;
            }
            vocab_free(&v);
        } else if (at->kind == HBGEN_ZIPF) {
            double* cdf = zipf_cdf(at->n_values, at->zipf_s);
            for (uint32_t i = 0; i < nb; ++i) iv[(size_t)i * na + a] = zipf_draw(&r, cdf, at->n_values);
            free(cdf);
            if (at->cap > 0) {
                /* split over-full values into codes of <= cap base tuples */
                uint32_t* seen = (uint32_t*)calloc(at->n_values, sizeof(uint32_t));
                uint32_t* cnt = (uint32_t*)calloc(at->n_values, sizeof(uint32_t));
                int64_t* first_extra = (int64_t*)malloc(sizeof(int64_t) * at->n_values);
                for (uint32_t i = 0; i < nb; ++i) cnt[iv[(size_t)i * na + a]]++;
                int64_t next = at->n_values;
                for (uint32_t v = 0; v < at->n_values; ++v) {
                    first_extra[v] = next;
                    if (cnt[v] > at->cap) next += (cnt[v] + at->cap - 1) / at->cap - 1;
                }
                for (uint32_t i = 0; i < nb; ++i) {
                    int64_t v = iv[(size_t)i * na + a];
                    uint32_t k = seen[v]++ / at->cap;
                    if (k > 0) iv[(size_t)i * na + a] = first_extra[v] + (k - 1);
                }
                free(seen); free(cnt); free(first_extra);
            }
        } else if (at->kind == HBGEN_CODES) {
            int64_t* codes = (int64_t*)malloc(sizeof(int64_t) * at->n_values);
            uint64_t span = (uint64_t)(at->hi - at->lo) + 1;
            for (uint32_t v = 0; v < at->n_values; ++v) {
                for (;;) {
                    int64_t c = at->lo + (int64_t)xo_below(&r, span);
                    int dupc = 0;
                    for (uint32_t u = 0; u < v; ++u) if (codes[u] == c) { dupc = 1; break; }
                    if (!dupc) { codes[v] = c; break; }
                }
            }
            for (uint32_t i = 0; i < nb; ++i) iv[(size_t)i * na + a] = codes[xo_below(&r, at->n_values)];
            free(codes);
        } else {
            uint64_t span = (uint64_t)(at->hi - at->lo) + 1;
            for (uint32_t i = 0; i < nb; ++i) iv[(size_t)i * na + a] = at->lo + (int64_t)xo_below(&r, span);
        }
    }

    /* duplicates */
    {
        xo256 r; xo_seed(&r, attr_seed(spec->seed, 0xD0D0u));
        uint32_t n_edit = 0;
        uint32_t edit_attrs[256];
        for (uint32_t a = 0; a < na && n_edit < 256; ++a)
            if ((attrs[a].kind == HBGEN_STRING || attrs[a].kind == HBGEN_WORDS || attrs[a].kind == HBGEN_KEYED) &&
                attrs[a].editable)
                edit_attrs[n_edit++] = a;
        for (uint32_t d = 0; d < nd; ++d) {
            uint32_t i = nb + d;
            uint32_t s = (uint32_t)xo_below(&r, nb);
            src[i] = s;
            for (uint32_t a = 0; a < na; ++a) {
                if (attrs[a].kind == HBGEN_STRING || attrs[a].kind == HBGEN_WORDS || attrs[a].kind == HBGEN_KEYED) {
                    sbuf b = sv[(size_t)s * na + a];
                    char* p = (char*)malloc(b.len + spec->edit_max + 1);
                    memcpy(p, b.p, b.len);
                    sv[(size_t)i * na + a].p = p; sv[(size_t)i * na + a].len = b.len;
                } else {
                    iv[(size_t)i * na + a] = iv[(size_t)s * na + a];
                }
            }
            uint32_t E = spec->edit_min + (uint32_t)xo_below(&r, (uint64_t)(spec->edit_max - spec->edit_min) + 1);
            for (uint32_t e = 0; e < E && n_edit > 0; ++e) {
                uint32_t a = edit_attrs[xo_below(&r, n_edit)];
                const char* al = ALPHA[attrs[a].kind == HBGEN_WORDS ? 2 : attrs[a].alphabet];
                uint32_t asz = (uint32_t)strlen(al);
                sbuf* b = &sv[(size_t)i * na + a];
                uint32_t type = (uint32_t)xo_below(&r, 3);
                if (b->len == 0) type = 1; /* only an insertion applies to an empty string */
                if (type == 0) {          /* substitute */
                    uint32_t pos = (uint32_t)xo_below(&r, b->len);
                    b->p[pos] = al[xo_below(&r, asz)];
                } else if (type == 1) {   /* insert */
                    uint32_t pos = (uint32_t)xo_below(&r, (uint64_t)b->len + 1);
                    memmove(b->p + pos + 1, b->p + pos, b->len - pos);
                    b->p[pos] = al[xo_below(&r, asz)];
                    b->len++;
                } else {                  /* delete */
                    uint32_t pos = (uint32_t)xo_below(&r, b->len);
                    memmove(b->p + pos, b->p + pos + 1, b->len - pos - 1);
                    b->len--;
                }
            }
            for (uint32_t a = 0; a < na; ++a) {
                if (attrs[a].kind == HBGEN_INT && attrs[a].int_p > 0.0) {
                    if (xo_unit(&r) < attrs[a].int_p) {
                        int64_t delta = (int64_t)xo_below(&r, (uint64_t)(2 * attrs[a].int_d + 1)) - attrs[a].int_d;
                        iv[(size_t)i * na + a] += delta;
                    }
                }
            }
        }
        for (uint32_t i = 0; i < nb; ++i) src[i] = -1;
    }

    /* final row order: random permutation (Fisher-Yates) */
    uint32_t* perm = (uint32_t*)malloc(sizeof(uint32_t) * n);   /* perm[new] = staging row */
    uint32_t* inv = (uint32_t*)malloc(sizeof(uint32_t) * n);    /* inv[staging] = new row */
    {
        xo256 r; xo_seed(&r, attr_seed(spec->seed, 0x9E12u));
        for (uint32_t i = 0; i < n; ++i) perm[i] = i;
        for (uint32_t i = n - 1; i > 0; --i) {
            uint32_t j = (uint32_t)xo_below(&r, (uint64_t)i + 1);
            uint32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
        }
        for (uint32_t i = 0; i < n; ++i) inv[perm[i]] = i;
    }

    for (uint32_t a = 0; a < na && rc == 0; ++a) {
        if (attrs[a].kind == HBGEN_STRING || attrs[a].kind == HBGEN_WORDS || attrs[a].kind == HBGEN_KEYED) {
            uint64_t off = 0;
            out[a].offsets[0] = 0;
            for (uint32_t i = 0; i < n; ++i) {
                sbuf b = sv[(size_t)perm[i] * na + a];
                if (off + b.len > out[a].bytes_cap) { rc = -1; break; }
                memcpy(out[a].bytes + off, b.p, b.len);
                off += b.len;
                out[a].offsets[i + 1] = off;
            }
            bytes_used[a] = off;
        } else {
            for (uint32_t i = 0; i < n; ++i) out[a].values[i] = iv[(size_t)perm[i] * na + a];
            bytes_used[a] = 0;
        }
    }
    for (uint32_t i = 0; i < n; ++i) {
        int64_t s = src[perm[i]];
        dup_src[i] = s < 0 ? -1 : (int64_t)inv[s];
    }

    for (size_t k = 0; k < (size_t)n * na; ++k) free(sv[k].p);
    free(sv); free(iv); free(src); free(perm); free(inv);
    return rc;
}
