/* The oracle's functions run under AddressSanitizer and UndefinedBehaviorSanitizer on small inputs,
   with their three count statements cross-checked.  Exits non-zero on a disagreement. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int64_t or_rank_bits(const uint64_t *, uint64_t, const uint64_t *, uint64_t, uint64_t *);
int64_t or_rank_dna(const uint64_t *, uint64_t, const uint64_t *, const uint8_t *, uint64_t, uint64_t *);
int64_t or_rank4_dna(const uint64_t *, uint64_t, const uint64_t *, uint64_t, uint64_t *);
int64_t or_prefix_rank_dna(const uint64_t *, uint64_t, const uint64_t *, const uint8_t *, uint64_t, uint64_t *);
void or_count_naive(const uint8_t *, uint64_t, const uint8_t *, const uint64_t *, uint64_t, uint64_t *);
void or_suffix_array(const uint8_t *, uint64_t, int64_t *);
uint64_t or_bwt(const uint8_t *, uint64_t, const int64_t *, uint8_t *);
void or_count_sa(const uint8_t *, uint64_t, const int64_t *, const uint8_t *, const uint64_t *, uint64_t, uint64_t *);
int or_count_backward(const uint8_t *, uint64_t, const uint8_t *, const uint64_t *, uint64_t, uint64_t *);
int or_kmer_intervals(const uint8_t *, uint64_t, int, uint64_t *, uint64_t *);
void or_interval_sa(const uint8_t *, uint64_t, const int64_t *, const uint8_t *, const uint64_t *, uint64_t, uint64_t *,
                    uint64_t *);

static uint64_t mix(uint64_t x) {
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}

int main(void) {
    const uint64_t sizes[] = {0, 1, 2, 31, 32, 33, 65, 500, 3000};
    int fail = 0;
    for (size_t si = 0; si < sizeof sizes / sizeof sizes[0]; ++si) {
        const uint64_t n = sizes[si];
        uint8_t *t = malloc(n + 1);
        uint64_t *packed = calloc((n + 31) / 32 + 1, 8), *bits = calloc((n + 63) / 64 + 1, 8);
        for (uint64_t i = 0; i < n; ++i) {
            t[i] = (uint8_t)(mix(n * 131 + i % 23) & 3);  /* repetitive, so counts exceed 1 */
            packed[i / 32] |= (uint64_t)t[i] << (2 * (i % 32));
            bits[i / 64] |= (mix(i) & 1) << (i % 64);
        }
        const uint64_t nq = n + 3;
        uint64_t *q = malloc(nq * 8), *r = malloc(nq * 8), *r4 = malloc(nq * 32);
        uint8_t *c = malloc(nq);
        for (uint64_t i = 0; i < nq; ++i) {
            q[i] = i;  /* includes q = n + 1, n + 2: out of range */
            c[i] = (uint8_t)(i % 5);  /* includes c = 4: out of range */
        }
        or_rank_bits(bits, n, q, nq, r);
        or_rank_dna(packed, n, q, c, nq, r);
        or_prefix_rank_dna(packed, n, q, c, nq, r);
        or_rank4_dna(packed, n, q, nq, r4);
        int64_t *sa = malloc((n + 1) * 8);
        uint8_t *b = malloc(n + 1);
        or_suffix_array(t, n, sa);
        or_bwt(t, n, sa, b);
        /* patterns: every substring of length 1..6 starting at a few places, plus absent ones */
        uint8_t pat[4096];
        uint64_t off[600], np = 0, len = 0;
        off[0] = 0;
        for (uint64_t s = 0; s + 6 <= n && np < 400; s += (n / 60) + 1) {
            for (uint64_t m = 1; m <= 6 && np < 400; ++m) {
                memcpy(pat + len, t + s, m);
                len += m;
                off[++np] = len;
            }
        }
        pat[len] = 4;  /* a code above 3 */
        len += 1;
        off[++np] = len;
        off[np + 1] = len;  /* the empty pattern */
        ++np;
        uint64_t *a1 = malloc(np * 8), *a2 = malloc(np * 8), *a3 = malloc(np * 8), *lo = malloc(np * 8),
                 *hi = malloc(np * 8);
        or_count_naive(t, n, pat, off, np, a1);
        or_count_sa(t, n, sa, pat, off, np, a2);
        or_count_backward(b, n, pat, off, np, a3);
        or_interval_sa(t, n, sa, pat, off, np, lo, hi);
        for (uint64_t p = 0; p < np; ++p)
            if (a1[p] != a2[p] || a2[p] != a3[p] || hi[p] - lo[p] != a1[p]) ++fail;
        uint64_t *klo = malloc((1u << 8) * 8), *khi = malloc((1u << 8) * 8);
        or_kmer_intervals(b, n, 4, klo, khi);
        free(klo), free(khi), free(a1), free(a2), free(a3), free(lo), free(hi);
        free(sa), free(b), free(q), free(r), free(r4), free(c), free(t), free(packed), free(bits);
    }
    printf("oracle: %d disagreements\n", fail);
    return fail ? 1 : 0;
}
