// Host-side FM-index input preparation: suffix array of T$ by induced sorting (SA-IS, Nong, Zhang
// and Chan, "Two efficient algorithms for linear time suffix array construction", IEEE TC 2011),
// then the BWT with the sentinel stored by position (paper Appendix D: a single '$' handled by
// storing its position in the BWT; here it is stored as A and the rank of A is corrected).
//
// The suffix array is built once per text and is not on the query path.
#include <stdint.h>

#include <cstring>
#include <new>
#include <vector>

#include "../../include/quadrank.h"

namespace {

template <typename Idx>
struct Sais {
    // Classify positions: S-type (true) if suffix i < suffix i+1.  The last symbol is the unique
    // smallest sentinel, which is S-type.
    template <typename Ch>
    static void classify(const Ch *s, Idx n, std::vector<bool> &stype) {
        stype.assign((size_t)n, false);
        stype[(size_t)n - 1] = true;
        for (Idx i = n - 1; i-- > 0;) stype[i] = s[i] < s[i + 1] || (s[i] == s[i + 1] && stype[(size_t)i + 1]);
    }
    static bool is_lms(const std::vector<bool> &st, Idx i) { return i > 0 && st[(size_t)i] && !st[(size_t)i - 1]; }

    template <typename Ch>
    static void bucket_bounds(const Ch *s, Idx n, Idx K, std::vector<Idx> &bkt, bool ends) {
        std::vector<Idx> cnt((size_t)K, 0);
        for (Idx i = 0; i < n; ++i) cnt[(size_t)s[i]]++;
        bkt.assign((size_t)K, 0);
        Idx sum = 0;
        for (Idx c = 0; c < K; ++c) {
            sum += cnt[(size_t)c];
            bkt[(size_t)c] = ends ? sum : sum - cnt[(size_t)c];
        }
    }

    // Induce the order of L-type then S-type suffixes from the LMS suffixes already placed.
    template <typename Ch>
    static void induce(const Ch *s, Idx *SA, Idx n, Idx K, const std::vector<bool> &st) {
        std::vector<Idx> bkt;
        bucket_bounds(s, n, K, bkt, false);
        for (Idx i = 0; i < n; ++i) {
            Idx j = SA[i] - 1;
            if (SA[i] > 0 && !st[(size_t)j]) SA[bkt[(size_t)s[j]]++] = j;
        }
        bucket_bounds(s, n, K, bkt, true);
        for (Idx i = n; i-- > 0;) {
            Idx j = SA[i] - 1;
            if (SA[i] > 0 && st[(size_t)j]) SA[--bkt[(size_t)s[j]]] = j;
        }
    }

    // s[0..n) over alphabet [0, K), s[n-1] the unique smallest symbol.  Writes SA[0..n).
    template <typename Ch>
    static void run(const Ch *s, Idx *SA, Idx n, Idx K) {
        if (n == 1) {
            SA[0] = 0;
            return;
        }
        std::vector<bool> st;
        classify(s, n, st);
        std::vector<Idx> bkt;
        // Stage 1: sort the LMS substrings.
        bucket_bounds(s, n, K, bkt, true);
        for (Idx i = 0; i < n; ++i) SA[i] = -1;
        for (Idx i = 1; i < n; ++i)
            if (is_lms(st, i)) SA[--bkt[(size_t)s[i]]] = i;
        induce(s, SA, n, K, st);
        // Compact the sorted LMS positions into the front of SA.
        Idx m = 0;
        for (Idx i = 0; i < n; ++i)
            if (is_lms(st, SA[i])) SA[m++] = SA[i];
        // Name the LMS substrings: equal substrings get equal names.
        for (Idx i = m; i < n; ++i) SA[i] = -1;
        Idx name = 0, prev = -1;
        for (Idx i = 0; i < m; ++i) {
            Idx pos = SA[i];
            bool diff = prev < 0;
            for (Idx d = 0; !diff; ++d) {
                if (s[pos + d] != s[prev + d] || st[(size_t)(pos + d)] != st[(size_t)(prev + d)]) {
                    diff = true;
                } else if (d > 0 && (is_lms(st, pos + d) || is_lms(st, prev + d))) {
                    break;  // both substrings ended at an LMS position and were equal
                }
            }
            if (diff) {
                ++name;
                prev = pos;
            }
            SA[m + pos / 2] = name - 1;  // LMS positions are >= 2 apart, so pos/2 is unique
        }
        // Gather the reduced string in text order.
        Idx *s1 = SA + n - m;
        for (Idx i = n, j = n; i-- > m;)
            if (SA[i] >= 0) SA[--j] = SA[i];
        // Stage 2: sort the reduced problem (recursively if names repeat).
        std::vector<Idx> sa1((size_t)m);
        if (name < m) {
            std::vector<Idx> s1c(s1, s1 + m);
            run<Idx>(s1c.data(), sa1.data(), m, name);
        } else {
            for (Idx i = 0; i < m; ++i) sa1[(size_t)s1[i]] = i;
        }
        // Map reduced ranks back to LMS positions (text order of LMS positions).
        std::vector<Idx> lms;
        lms.reserve((size_t)m);
        for (Idx i = 1; i < n; ++i)
            if (is_lms(st, i)) lms.push_back(i);
        // Stage 3: place the LMS suffixes in sorted order at their bucket ends, then induce.
        bucket_bounds(s, n, K, bkt, true);
        for (Idx i = 0; i < n; ++i) SA[i] = -1;
        for (Idx i = m; i-- > 0;) {
            Idx j = lms[(size_t)sa1[(size_t)i]];
            SA[--bkt[(size_t)s[j]]] = j;
        }
        induce(s, SA, n, K, st);
    }
};

// BWT of T$ and, when rate > 0, the suffix-array sample for locate: row k is marked (bit k of
// mark_bits) iff SA[k] is a multiple of rate, and samples[] lists SA[k] of the marked rows in row
// order (positions 0, rate, 2 rate, ... <= n: floor(n/rate) + 1 of them).
template <typename Idx>
int bwt_from_text(const uint8_t *text, uint64_t n, uint64_t *bwt_packed, uint64_t *dollar_pos, uint32_t rate,
                  uint64_t *mark_bits, uint32_t *samples) {
    // s = text codes + 1 followed by the sentinel 0.
    std::vector<uint8_t> s;
    std::vector<Idx> SA;
    try {
        s.resize((size_t)n + 1);
        SA.resize((size_t)n + 1);
    } catch (const std::bad_alloc &) {
        return QR_ENOMEM;
    }
    for (uint64_t i = 0; i < n; ++i) s[i] = (uint8_t)(text[i] + 1);
    s[n] = 0;
    Sais<Idx>::run(s.data(), SA.data(), (Idx)(n + 1), (Idx)5);
    const uint64_t words = (n + 1 + 31) / 32;
    std::memset(bwt_packed, 0, words * 8);
    uint64_t dpos = 0;
    for (uint64_t k = 0; k <= n; ++k) {
        const Idx j = SA[k];
        uint64_t code = 0;  // '$' row stores A
        if (j == 0) dpos = k;
        else code = text[j - 1];
        bwt_packed[k / 32] |= code << (2 * (k % 32));
    }
    *dollar_pos = dpos;
    if (rate) {
        std::memset(mark_bits, 0, ((n + 1 + 63) / 64) * 8);
        uint64_t m = 0;
        for (uint64_t k = 0; k <= n; ++k) {
            const uint64_t j = (uint64_t)SA[k];
            if (j % rate == 0) {
                mark_bits[k / 64] |= 1ull << (k % 64);
                samples[m++] = (uint32_t)j;
            }
        }
    }
    return QR_OK;
}

}  // namespace

extern "C" int quadfm_index_host(const uint8_t *h_text, uint64_t n, uint32_t rate, uint64_t *h_bwt_packed2,
                                 uint64_t *dollar_pos, uint64_t *h_mark_bits, uint32_t *h_samples) {
    if ((!h_text && n) || !h_bwt_packed2 || !dollar_pos || (rate && (!h_mark_bits || !h_samples))) return QR_EINVAL;
    if (n + 1 > 0xffffffffull) return QR_ERANGE;  // the FM-index counts are u32 intervals
    for (uint64_t i = 0; i < n; ++i)
        if (h_text[i] > 3) return QR_EINVAL;
    if (n + 1 < 0x7fffffffull)
        return bwt_from_text<int32_t>(h_text, n, h_bwt_packed2, dollar_pos, rate, h_mark_bits, h_samples);
    return bwt_from_text<int64_t>(h_text, n, h_bwt_packed2, dollar_pos, rate, h_mark_bits, h_samples);
}

extern "C" int quadfm_bwt_host(const uint8_t *h_text, uint64_t n, uint64_t *h_bwt_packed2, uint64_t *dollar_pos) {
    return quadfm_index_host(h_text, n, 0, h_bwt_packed2, dollar_pos, nullptr, nullptr);
}
