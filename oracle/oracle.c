/*
 * ORACLE — test infrastructure only.
 *
 * A plain, slow, obviously correct CPU statement of what the GPU path
 * computes.  Only the tests, the smoke check and the benchmark's CPU-baseline
 * leg may load this library; the product never does.  It shares no code,
 * header, table or constant with the GPU library.
 *
 * Everything is exact integer arithmetic.  Input encoding (same documented
 * convention as the product's boundary): bit i of a bitvector is bit (i mod 64)
 * of u64 word i/64; DNA codes A=0, C=1, G=2, T=3 with base i in bits
 * [2(i mod 32), +2) of u64 word i/32.  Bits or bases beyond n are ignored.
 *
 * Sources (QuadRank paper, arXiv 2602.04103):
 *   rank definition ............ Section 1, display equation for rank(q,c);
 *                                Section 3 opening paragraph for rank(q)=rank(q,1)
 *   rank4 ...................... Section 4, first paragraph (all four symbols at once)
 *   FM-index count ............. Appendix D (count only, single direction, sentinel
 *                                by position, prefix lookup table for 8 characters)
 * Where the paper is silent (C array, sentinel order, edge patterns) the
 * textbook FM-index conventions are used: '$' sorts before A < C < G < T,
 * C[c] = 1 + number of text characters smaller than c, the search starts from
 * the interval [0, n+1) and an interval with sp >= ep is empty.
 */
#define _GNU_SOURCE /* qsort_r */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_BAD UINT64_MAX

#include <omp.h>

/* Threads of the OpenMP loops over queries from now on; returns the previous setting.  The loops'
   results do not depend on it (each query is answered on its own). */
int or_set_threads(int n) {
    int prev = omp_get_max_threads();
    if (n > 0) omp_set_num_threads(n);
    return prev;
}

/* ---- binary rank: rank(q) = #{ i < q : t_i = 1 }, 0 <= q <= n ---------------------------------- */

static uint64_t word_masked(const uint64_t *words, uint64_t n, uint64_t w) {
    /* word w with the bits at positions >= n cleared */
    uint64_t x = words[w];
    uint64_t first = w * 64;
    if (first + 64 > n) {
        uint64_t keep = n - first; /* 0..63 */
        x = keep ? (x & ((1ULL << keep) - 1ULL)) : 0;
    }
    return x;
}

/* out[i] = rank(q[i]); returns the number of queries with q > n (their output is UINT64_MAX). */
int64_t or_rank_bits(const uint64_t *words, uint64_t n, const uint64_t *q, uint64_t nq, uint64_t *out) {
    uint64_t nw = (n + 63) / 64;
    /* W[k] = number of 1 bits in words 0..k-1 (bits < n only) */
    uint64_t *W = (uint64_t *)malloc((nw + 1) * sizeof(uint64_t));
    if (!W) return -1;
    W[0] = 0;
    for (uint64_t k = 0; k < nw; ++k) W[k + 1] = W[k] + (uint64_t)__builtin_popcountll(word_masked(words, n, k));
    int64_t bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (int64_t i = 0; i < (int64_t)nq; ++i) {
        uint64_t p = q[i];
        if (p > n) {
            out[i] = OR_BAD;
            bad++;
            continue;
        }
        uint64_t k = p / 64, r = p % 64;
        uint64_t v = W[k];
        if (r) v += (uint64_t)__builtin_popcountll(words[k] & ((1ULL << r) - 1ULL));
        out[i] = v;
    }
    free(W);
    return bad;
}

/* ---- DNA rank: rank(q,c) = #{ i < q : t_i = c } and rank4(q) = (rank(q,0..3)) ------------------ */

static inline unsigned base_at(const uint64_t *packed, uint64_t i) {
    return (unsigned)((packed[i / 32] >> (2 * (i % 32))) & 3u);
}

/* W4[4k + c] = number of bases equal to c among positions [0, 32k) (positions < n only). */
static uint64_t *dna_prefix(const uint64_t *packed, uint64_t n, uint64_t *nw_out) {
    uint64_t nw = (n + 31) / 32;
    uint64_t *W = (uint64_t *)malloc(4 * (nw + 1) * sizeof(uint64_t));
    if (!W) return NULL;
    for (int c = 0; c < 4; ++c) W[c] = 0;
    for (uint64_t k = 0; k < nw; ++k) {
        uint64_t cnt[4] = {0, 0, 0, 0};
        for (uint64_t i = 32 * k; i < 32 * k + 32 && i < n; ++i) cnt[base_at(packed, i)]++;
        for (int c = 0; c < 4; ++c) W[4 * (k + 1) + c] = W[4 * k + c] + cnt[c];
    }
    *nw_out = nw;
    return W;
}

int64_t or_rank_dna(const uint64_t *packed, uint64_t n, const uint64_t *q, const uint8_t *c, uint64_t nq,
                    uint64_t *out) {
    uint64_t nw;
    uint64_t *W = dna_prefix(packed, n, &nw);
    if (!W) return -1;
    int64_t bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (int64_t i = 0; i < (int64_t)nq; ++i) {
        uint64_t p = q[i];
        unsigned s = c[i];
        if (p > n || s > 3) {
            out[i] = OR_BAD;
            bad++;
            continue;
        }
        uint64_t k = p / 32, v = W[4 * k + s];
        for (uint64_t j = 32 * k; j < p; ++j) v += (base_at(packed, j) == s);
        out[i] = v;
    }
    free(W);
    return bad;
}

int64_t or_rank4_dna(const uint64_t *packed, uint64_t n, const uint64_t *q, uint64_t nq, uint64_t *out4) {
    uint64_t nw;
    uint64_t *W = dna_prefix(packed, n, &nw);
    if (!W) return -1;
    int64_t bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (int64_t i = 0; i < (int64_t)nq; ++i) {
        uint64_t p = q[i];
        if (p > n) {
            for (int s = 0; s < 4; ++s) out4[4 * i + s] = OR_BAD;
            bad++;
            continue;
        }
        uint64_t k = p / 32, v[4];
        for (int s = 0; s < 4; ++s) v[s] = W[4 * k + s];
        for (uint64_t j = 32 * k; j < p; ++j) v[base_at(packed, j)]++;
        for (int s = 0; s < 4; ++s) out4[4 * i + s] = v[s];
    }
    free(W);
    return bad;
}

/* prefix_rank(q, c) = #{ i < q : t_i <= c }, the count of characters at most c (the operation the
   paper's closing section names for a bidirectional FM-index), over the same per-word prefix counts. */
int64_t or_prefix_rank_dna(const uint64_t *packed, uint64_t n, const uint64_t *q, const uint8_t *c, uint64_t nq,
                           uint64_t *out) {
    uint64_t nw;
    uint64_t *W = dna_prefix(packed, n, &nw);
    if (!W) return -1;
    int64_t bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (int64_t i = 0; i < (int64_t)nq; ++i) {
        uint64_t p = q[i];
        unsigned s = c[i];
        if (p > n || s > 3) {
            out[i] = OR_BAD;
            bad++;
            continue;
        }
        uint64_t k = p / 32, v = 0;
        for (unsigned x = 0; x <= s; ++x) v += W[4 * k + x];
        for (uint64_t j = 32 * k; j < p; ++j) v += (base_at(packed, j) <= s);
        out[i] = v;
    }
    free(W);
    return bad;
}

/* ---- FM-index count ------------------------------------------------------------------------------ */

/* count(P) = #{ i in [0, n-m] : T[i..i+m) = P } by direct comparison at every start.  A pattern
   code > 3 cannot match an ACGT text; m = 0 gives n+1 (every position 0..n, the FM full interval). */
void or_count_naive(const uint8_t *text, uint64_t n, const uint8_t *pat, const uint64_t *off, uint64_t npat,
                    uint64_t *out) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < (int64_t)npat; ++p) {
        const uint8_t *P = pat + off[p];
        uint64_t m = off[p + 1] - off[p], cnt = 0;
        if (m == 0) {
            out[p] = n + 1;
            continue;
        }
        if (m <= n) {
            for (uint64_t i = 0; i + m <= n; ++i) {
                if (text[i] == P[0] && memcmp(text + i, P, m) == 0) cnt++;
            }
        }
        out[p] = cnt;
    }
}

/* Suffix array of T$ (n+1 suffixes, '$' at position n sorting first) by plain comparison sort. */
static int cmp_suffix(const void *a, const void *b, void *ctx) {
    const uint8_t *T = ((const uint8_t **)ctx)[0];
    uint64_t n = (uint64_t)(uintptr_t)((const uint8_t **)ctx)[1];
    int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
    while ((uint64_t)i < n && (uint64_t)j < n) {
        if (T[i] != T[j]) return T[i] < T[j] ? -1 : 1;
        ++i;
        ++j;
    }
    /* the suffix that reaches '$' first is the smaller one */
    if ((uint64_t)i == n && (uint64_t)j == n) return 0;
    return (uint64_t)i == n ? -1 : 1;
}

void or_suffix_array(const uint8_t *text, uint64_t n, int64_t *sa) {
    for (uint64_t i = 0; i <= n; ++i) sa[i] = (int64_t)i;
    const uint8_t *ctx[2] = {text, (const uint8_t *)(uintptr_t)n};
    qsort_r(sa, n + 1, sizeof(int64_t), cmp_suffix, (void *)ctx);
}

/* Check a suffix array of T$ given as n+1 row values, without building one: it must be a
   permutation of 0..n, and each pair of neighbouring rows must hold two suffixes in strictly
   increasing order, compared character by character with the end of the text ('$') smaller than
   any character (the same order the comparison sort above uses).  Returns 0 if both hold, 1 if a
   value is out of range or repeated (some row is then missing), 2 if a neighbouring pair is out of
   order, -1 if memory runs out. */
int or_check_sa(const uint8_t *text, uint64_t n, const int64_t *sa) {
    uint64_t nw = (n + 1 + 63) / 64;
    uint64_t *seen = (uint64_t *)calloc(nw, sizeof(uint64_t));
    if (!seen) return -1;
    int bad = 0;
    for (uint64_t k = 0; k <= n && !bad; ++k) {
        int64_t v = sa[k];
        if (v < 0 || (uint64_t)v > n || (seen[(uint64_t)v / 64] >> ((uint64_t)v % 64) & 1)) bad = 1;
        else seen[(uint64_t)v / 64] |= 1ULL << ((uint64_t)v % 64);
    }
    free(seen);
    if (bad) return 1;
    int disorder = 0;
#pragma omp parallel for schedule(static) reduction(| : disorder)
    for (int64_t k = 0; k < (int64_t)n; ++k) {
        uint64_t i = (uint64_t)sa[k], j = (uint64_t)sa[k + 1];
        while (i < n && j < n && text[i] == text[j]) {
            ++i;
            ++j;
        }
        /* suffix i < suffix j iff i reached the end first, or both go on and T[i] < T[j] */
        int less = (i == n && j < n) || (i < n && j < n && text[i] < text[j]);
        disorder |= !less;
    }
    return disorder ? 2 : 0;
}

/* BWT[k] = T[SA[k]-1], or '$' (code 4 here) where SA[k] = 0.  Returns the row of '$'. */
uint64_t or_bwt(const uint8_t *text, uint64_t n, const int64_t *sa, uint8_t *bwt) {
    uint64_t dollar = 0;
    for (uint64_t k = 0; k <= n; ++k) {
        if (sa[k] == 0) {
            bwt[k] = 4;
            dollar = k;
        } else {
            bwt[k] = text[sa[k] - 1];
        }
    }
    return dollar;
}

/* compare the first m characters of suffix i with P: <0, 0 (P is a prefix), >0 */
static int cmp_prefix(const uint8_t *T, uint64_t n, uint64_t i, const uint8_t *P, uint64_t m) {
    for (uint64_t t = 0; t < m; ++t) {
        if (i + t >= n) return -1; /* suffix ended ('$' is smallest) */
        if (T[i + t] != P[t]) return T[i + t] < P[t] ? -1 : 1;
    }
    return 0;
}

/* The SA range [lo, hi) of the suffixes that start with P, by binary search; [0, 0) when P holds
   a code > 3 (it cannot occur in an ACGT text). */
void or_interval_sa(const uint8_t *text, uint64_t n, const int64_t *sa, const uint8_t *pat, const uint64_t *off,
                    uint64_t npat, uint64_t *lo_out, uint64_t *hi_out) {
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < (int64_t)npat; ++p) {
        const uint8_t *P = pat + off[p];
        uint64_t m = off[p + 1] - off[p];
        int bad = 0;
        for (uint64_t t = 0; t < m; ++t) bad |= P[t] > 3;
        if (bad) {
            lo_out[p] = hi_out[p] = 0;
            continue;
        }
        /* lo = first k with suffix(SA[k]) >= P (prefix-wise); hi = first k with suffix > P */
        uint64_t a = 0, b = n + 1;
        while (a < b) {
            uint64_t mid = a + (b - a) / 2;
            if (cmp_prefix(text, n, (uint64_t)sa[mid], P, m) < 0) a = mid + 1; else b = mid;
        }
        uint64_t lo = a;
        b = n + 1;
        while (a < b) {
            uint64_t mid = a + (b - a) / 2;
            if (cmp_prefix(text, n, (uint64_t)sa[mid], P, m) <= 0) a = mid + 1; else b = mid;
        }
        lo_out[p] = lo;
        hi_out[p] = a;
    }
}

/* count = size of that SA range */
void or_count_sa(const uint8_t *text, uint64_t n, const int64_t *sa, const uint8_t *pat, const uint64_t *off,
                 uint64_t npat, uint64_t *out) {
    uint64_t *lo = (uint64_t *)malloc((npat ? npat : 1) * sizeof(uint64_t));
    if (!lo) abort();
    or_interval_sa(text, n, sa, pat, off, npat, lo, out);
    for (uint64_t p = 0; p < npat; ++p) out[p] -= lo[p];
    free(lo);
}

/* Textbook backward search over a BWT in which '$' is its own symbol (code 4).
   occ(q, c) = #{k < q : BWT[k] = c} is answered from a prefix count every 64 rows plus a loop. */
typedef struct {
    const uint8_t *bwt;
    uint64_t len; /* n + 1 */
    uint64_t *S;  /* S[5*b + c] = occurrences of c in rows [0, 64b) */
    uint64_t C[5];
} occ_t;

static int occ_init(occ_t *o, const uint8_t *bwt, uint64_t n) {
    o->bwt = bwt;
    o->len = n + 1;
    uint64_t nb = o->len / 64 + 1;
    o->S = (uint64_t *)calloc(5 * (nb + 1), sizeof(uint64_t));
    if (!o->S) return -1;
    uint64_t cnt[5] = {0, 0, 0, 0, 0};
    for (uint64_t k = 0; k < o->len; ++k) {
        if (k % 64 == 0)
            for (int c = 0; c < 5; ++c) o->S[5 * (k / 64) + c] = cnt[c];
        cnt[bwt[k]]++;
    }
    if (o->len % 64 == 0)
        for (int c = 0; c < 5; ++c) o->S[5 * (o->len / 64) + c] = cnt[c];
    /* C[c] = 1 ('$') + number of text characters smaller than c */
    uint64_t acc = 1;
    for (int c = 0; c < 4; ++c) {
        o->C[c] = acc;
        acc += cnt[c];
    }
    return 0;
}

static uint64_t occ(const occ_t *o, uint64_t q, unsigned c) {
    uint64_t v = o->S[5 * (q / 64) + c];
    for (uint64_t k = (q / 64) * 64; k < q; ++k) v += (o->bwt[k] == c);
    return v;
}

static void backward(const occ_t *o, const uint8_t *P, uint64_t m, uint64_t *sp_io, uint64_t *ep_io) {
    uint64_t sp = *sp_io, ep = *ep_io;
    for (uint64_t t = m; t-- > 0;) {
        if (sp >= ep) break;
        unsigned c = P[t];
        if (c > 3) {
            sp = ep = 0;
            break;
        }
        sp = o->C[c] + occ(o, sp, c);
        ep = o->C[c] + occ(o, ep, c);
    }
    *sp_io = sp;
    *ep_io = ep;
}

int or_count_backward(const uint8_t *bwt, uint64_t n, const uint8_t *pat, const uint64_t *off, uint64_t npat,
                      uint64_t *out) {
    occ_t o;
    if (occ_init(&o, bwt, n)) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < (int64_t)npat; ++p) {
        uint64_t sp = 0, ep = n + 1;
        backward(&o, pat + off[p], off[p + 1] - off[p], &sp, &ep);
        out[p] = ep > sp ? ep - sp : 0;
    }
    free(o.S);
    return 0;
}

/* Interval [lo, hi) after k backward steps over every k-mer w (first character most significant,
   the last character processed first), starting from [0, n+1). */
int or_kmer_intervals(const uint8_t *bwt, uint64_t n, int k, uint64_t *lo, uint64_t *hi) {
    occ_t o;
    if (occ_init(&o, bwt, n)) return -1;
    uint64_t nk = 1ULL << (2 * k);
#pragma omp parallel for schedule(static)
    for (int64_t w = 0; w < (int64_t)nk; ++w) {
        uint8_t P[32];
        for (int t = 0; t < k; ++t) P[t] = (uint8_t)(((uint64_t)w >> (2 * (k - 1 - t))) & 3u);
        uint64_t sp = 0, ep = n + 1;
        backward(&o, P, (uint64_t)k, &sp, &ep);
        lo[w] = sp;
        hi[w] = ep;
    }
    free(o.S);
    return 0;
}
