// Host input preparation (suffix array by induced sorting, BWT, suffix-array sample) run under
// AddressSanitizer and UndefinedBehaviorSanitizer on texts of many sizes and shapes.  Exits non-zero
// when an output is inconsistent; the sanitizers abort on any memory or undefined-behaviour error.
#include <cstdint>
#include <cstdio>
#include <vector>

extern "C" int quadfm_index_host(const uint8_t *h_text, uint64_t n, uint32_t rate, uint64_t *h_bwt_packed2,
                                 uint64_t *dollar_pos, uint64_t *h_mark_bits, uint32_t *h_samples);

static uint64_t mix(uint64_t x) {  // SplitMix64 finaliser
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}

static int check(const std::vector<uint8_t> &t, uint32_t rate) {
    const uint64_t n = t.size();
    std::vector<uint64_t> bwt((n + 1 + 31) / 32 + 1), marks((n + 1 + 63) / 64 + 1);
    std::vector<uint32_t> samples(rate ? n / rate + 1 : 1);
    uint64_t dollar = ~0ull;
    if (quadfm_index_host(t.data(), n, rate, bwt.data(), &dollar, marks.data(), samples.data()) != 0) return 1;
    if (dollar > n) return 2;
    uint64_t want[4] = {0, 0, 0, 0}, got[4] = {0, 0, 0, 0};
    for (uint8_t c : t) want[c]++;
    for (uint64_t k = 0; k <= n; ++k)
        if (k != dollar) got[(bwt[k / 32] >> (2 * (k % 32))) & 3]++;
    for (int c = 0; c < 4; ++c)
        if (got[c] != want[c]) return 3;  // the BWT is a permutation of the text plus '$'
    if (rate) {
        uint64_t m = 0;
        for (uint64_t k = 0; k <= n; ++k) m += (marks[k / 64] >> (k % 64)) & 1;
        if (m != n / rate + 1 || !((marks[dollar / 64] >> (dollar % 64)) & 1)) return 4;
        std::vector<uint8_t> seen(n + 1, 0);
        for (uint32_t s : samples) {
            if (s > n || s % rate || seen[s]) return 5;  // each multiple of rate exactly once
            seen[s] = 1;
        }
    }
    return 0;
}

int main() {
    const uint64_t sizes[] = {0, 1, 2, 3, 5, 31, 32, 33, 64, 100, 1000, 4097, 20000};
    uint64_t seed = 1;
    int failures = 0;
    for (uint64_t n : sizes) {
        for (int kind = 0; kind < 5; ++kind) {
            std::vector<uint8_t> t(n);
            for (uint64_t i = 0; i < n; ++i) {
                switch (kind) {
                    case 0: t[i] = (uint8_t)(mix(seed + i) & 3); break;                // random
                    case 1: t[i] = 0; break;                                          // all A
                    case 2: t[i] = 3; break;                                          // all T
                    case 3: t[i] = (uint8_t)(i % 7 % 4); break;                       // periodic
                    default: t[i] = (uint8_t)(mix(seed + (i % 37)) & 3); break;       // tiled repeat
                }
            }
            ++seed;
            for (uint32_t rate : {0u, 1u, 7u, 32u}) {
                const int r = check(t, rate);
                if (r) {
                    std::printf("inconsistent output: n=%llu kind=%d rate=%u code=%d\n", (unsigned long long)n, kind,
                                rate, r);
                    ++failures;
                }
            }
        }
    }
    const uint8_t bad[4] = {0, 1, 4, 2};  // a code above 3 is rejected, not read past
    uint64_t b[2], d;
    if (quadfm_index_host(bad, 4, 0, b, &d, nullptr, nullptr) == 0) ++failures;
    std::printf("host input preparation: %d failures\n", failures);
    return failures ? 1 : 0;
}
