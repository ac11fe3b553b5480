/*
 * Seeded synthetic inputs for the rank structures and the FM-index.
 *
 * This module holds only input generation and the documented input encoding
 * (2-bit packing).  It contains none of the rank / FM arithmetic; both the
 * oracle and the GPU path consume what it produces.
 *
 * Randomness: every draw is the i-th output of SplitMix64 (Steele, Lea and
 * Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014),
 * evaluated counter-style so any draw can be recomputed independently:
 *     x_i = mix(seed + (i + 1) * 0x9e3779b97f4a7c15)
 * with mix = the published variant-13 finaliser.  Independent streams for the
 * different purposes are obtained by re-seeding with mix(seed ^ tag * K).
 *
 * Input encoding (shared convention, not method arithmetic):
 *   - bit i of a bitvector = bit (i mod 64) of little-endian u64 word i/64;
 *   - DNA codes A=0, C=1, G=2, T=3; base i occupies bits [2(i mod 32), +2)
 *     of u64 word i/32.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN 0x9e3779b97f4a7c15ULL

static inline uint64_t sm_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* i-th SplitMix64 output for a seed (counter form). */
uint64_t dg_draw(uint64_t seed, uint64_t i) { return sm_mix(seed + (i + 1) * GOLDEN); }

/* Seed of an independent stream `tag` derived from `seed`. */
uint64_t dg_stream(uint64_t seed, uint64_t tag) { return sm_mix(seed ^ (tag * 0xd6e8feb86659fd93ULL + 0x632be59bd9b4e019ULL)); }

/* Uniform integer in [0, m) by 128-bit multiply-shift of a 64-bit draw. */
static inline uint64_t mulhi_range(uint64_t x, uint64_t m) {
    return (uint64_t)(((unsigned __int128)x * (unsigned __int128)m) >> 64);
}
uint64_t dg_range(uint64_t x, uint64_t m) { return mulhi_range(x, m); }

/* Uniform double in [0,1) from the top 53 bits of a draw. */
static inline double unit_double(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }

/*
 * Bernoulli bitvector: nwords u64 words.  thr16 in [0, 65536] is the success
 * threshold on 16-bit fields, P(bit=1) = thr16 / 65536.  thr16 == 32768 uses
 * one full 64-bit draw per word (exactly Bernoulli(1/2) per bit).
 */
void dg_bits(uint64_t seed, uint32_t thr16, uint64_t nwords, uint64_t *out) {
    if (thr16 == 32768u) {
#pragma omp parallel for schedule(static)
        for (int64_t w = 0; w < (int64_t)nwords; ++w) out[w] = dg_draw(seed, (uint64_t)w);
        return;
    }
#pragma omp parallel for schedule(static)
    for (int64_t w = 0; w < (int64_t)nwords; ++w) {
        uint64_t word = 0;
        for (int d = 0; d < 16; ++d) {
            uint64_t x = dg_draw(seed, (uint64_t)w * 16u + (uint64_t)d);
            for (int f = 0; f < 4; ++f) {
                uint32_t u = (uint32_t)((x >> (16 * f)) & 0xffffu);
                if (u < thr16) word |= 1ULL << (4 * d + f);
            }
        }
        out[w] = word;
    }
}

/* iid uniform DNA codes (one byte per base).  Base i is 2-bit field i%32 of draw i/32. */
void dg_dna_codes(uint64_t seed, uint64_t n, uint8_t *codes) {
    int64_t nw = (int64_t)((n + 31) / 32);
#pragma omp parallel for schedule(static)
    for (int64_t w = 0; w < nw; ++w) {
        uint64_t x = dg_draw(seed, (uint64_t)w);
        uint64_t base = (uint64_t)w * 32u;
        for (int k = 0; k < 32 && base + (uint64_t)k < n; ++k) codes[base + k] = (uint8_t)((x >> (2 * k)) & 3u);
    }
}

/*
 * Planted repeats: nseg source segments of length seglen are drawn (start
 * uniform in [0, n-seglen]) from the text as it is before planting; then each
 * segment is copied `copies` times, in seeded order, to a uniform start in
 * [0, n-seglen], later copies overwriting earlier ones.  Every copied base is
 * independently substituted with probability `sub` by a uniformly chosen
 * different base.  Returns 0, or -1 if the text is too short / allocation fails.
 */
int dg_plant_repeats(uint64_t seed, uint8_t *codes, uint64_t n, uint64_t nseg, uint64_t seglen,
                     uint64_t copies, double sub) {
    if (nseg == 0 || copies == 0) return 0;
    if (seglen == 0 || seglen > n) return -1;
    uint8_t *src = (uint8_t *)malloc(nseg * seglen);
    if (!src) return -1;
    uint64_t s_src = dg_stream(seed, 1), s_dst = dg_stream(seed, 2), s_sub = dg_stream(seed, 3);
    uint64_t span = n - seglen + 1;
    for (uint64_t s = 0; s < nseg; ++s) {
        uint64_t st = mulhi_range(dg_draw(s_src, s), span);
        memcpy(src + s * seglen, codes + st, seglen);
    }
    for (uint64_t s = 0; s < nseg; ++s) {
        for (uint64_t k = 0; k < copies; ++k) {
            uint64_t cid = s * copies + k;
            uint64_t dst = mulhi_range(dg_draw(s_dst, cid), span);
            const uint8_t *seg = src + s * seglen;
            for (uint64_t t = 0; t < seglen; ++t) {
                uint8_t b = seg[t];
                uint64_t x = dg_draw(s_sub, cid * seglen + t);
                if (unit_double(x) < sub) b = (uint8_t)((b + 1u + (uint8_t)mulhi_range(x << 11 | (x >> 53), 3)) & 3u);
                codes[dst + t] = b;
            }
        }
    }
    free(src);
    return 0;
}

/*
 * Pack codes into the 2-bit word layout.  Bits beyond n in the last word are
 * zero, or (tail_garbage_seed != 0) random junk, to exercise consumers that
 * must ignore them.
 */
void dg_pack2(const uint8_t *codes, uint64_t n, uint64_t tail_garbage_seed, uint64_t *words) {
    int64_t nw = (int64_t)((n + 31) / 32);
#pragma omp parallel for schedule(static)
    for (int64_t w = 0; w < nw; ++w) {
        uint64_t base = (uint64_t)w * 32u, x = 0;
        for (int k = 0; k < 32; ++k) {
            if (base + (uint64_t)k < n) x |= (uint64_t)(codes[base + k] & 3u) << (2 * k);
        }
        words[w] = x;
    }
    if (tail_garbage_seed && (n % 32)) {
        uint64_t keep = (1ULL << (2 * (n % 32))) - 1ULL;
        words[nw - 1] = (words[nw - 1] & keep) | (dg_draw(tail_garbage_seed, 0) & ~keep);
    }
}

/* Fill bits >= n of the last word with junk (bitvector form). */
void dg_bits_tail_garbage(uint64_t *words, uint64_t n, uint64_t seed) {
    if (n % 64 == 0) return;
    uint64_t keep = (1ULL << (n % 64)) - 1ULL;
    words[n / 64] = (words[n / 64] & keep) | (dg_draw(seed, 0) & ~keep);
}

/* Queries q_i uniform in [0, n] (inclusive): multiply-shift of draw i onto n+1 values. */
void dg_queries(uint64_t seed, uint64_t n, uint64_t nq, uint64_t *q) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)nq; ++i) q[i] = mulhi_range(dg_draw(seed, (uint64_t)i), n + 1);
}

/* Symbols c_i uniform in {0,1,2,3}: top two bits of draw i. */
void dg_symbols(uint64_t seed, uint64_t nq, uint8_t *c) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)nq; ++i) c[i] = (uint8_t)(dg_draw(seed, (uint64_t)i) >> 62);
}

/*
 * Pattern lengths uniform in [minlen, maxlen]; writes CSR offsets off[0..npat]
 * and returns the total number of characters.
 */
uint64_t dg_pattern_offsets(uint64_t seed, uint64_t npat, uint64_t minlen, uint64_t maxlen, uint64_t *off) {
    uint64_t s_len = dg_stream(seed, 11), acc = 0;
    off[0] = 0;
    for (uint64_t p = 0; p < npat; ++p) {
        acc += minlen + mulhi_range(dg_draw(s_len, p), maxlen - minlen + 1);
        off[p + 1] = acc;
    }
    return acc;
}

/*
 * Pattern contents.  Pattern p (length m = off[p+1]-off[p]) is, with
 * probability frac_sampled, the text window starting uniform in [0, n-m]
 * with per-base substitution probability `sub` (uniform different base);
 * otherwise iid uniform bases.  If m > n, the pattern is always iid.
 * kind[p] (optional) records 1 for sampled, 0 for iid.
 */
void dg_pattern_fill(uint64_t seed, const uint8_t *codes, uint64_t n, uint64_t npat, const uint64_t *off,
                     double frac_sampled, double sub, uint8_t *pat, uint8_t *kind) {
    uint64_t s_kind = dg_stream(seed, 12), s_pos = dg_stream(seed, 13), s_sub = dg_stream(seed, 14),
             s_iid = dg_stream(seed, 15);
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t pi = 0; pi < (int64_t)npat; ++pi) {
        uint64_t p = (uint64_t)pi, o = off[p], m = off[p + 1] - off[p];
        int sampled = (m <= n) && unit_double(dg_draw(s_kind, p)) < frac_sampled;
        if (kind) kind[p] = (uint8_t)sampled;
        if (sampled) {
            uint64_t st = mulhi_range(dg_draw(s_pos, p), n - m + 1);
            for (uint64_t t = 0; t < m; ++t) {
                uint8_t b = codes[st + t];
                uint64_t x = dg_draw(s_sub, o + t);
                if (unit_double(x) < sub) b = (uint8_t)((b + 1u + (uint8_t)mulhi_range(x << 11 | (x >> 53), 3)) & 3u);
                pat[o + t] = b;
            }
        } else {
            for (uint64_t t = 0; t < m; ++t) pat[o + t] = (uint8_t)(dg_draw(s_iid, o + t) >> 62);
        }
    }
}
