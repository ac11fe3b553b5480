// Device-side QuadRank query primitives (layout described in quadrank.hip), shared by the rank
// kernels and the FM-index search.
#pragma once

#include "common.hpp"

namespace qr {

// v.{x,y,z,w}[c] by mask arithmetic: a runtime-indexed select chain would be lowered to a
// stack array (scratch memory) once several queries are unrolled per lane.
__device__ __forceinline__ uint32_t sel4(const uint4 &v, uint32_t c) {
    const uint32_t m1 = 0u - (c & 1u), m2 = 0u - ((c >> 1) & 1u);
    const uint32_t lo = (v.x & ~m1) | (v.y & m1), hi = (v.z & ~m1) | (v.w & m1);
    return (lo & ~m2) | (hi & m2);
}

// ---- layouts -------------------------------------------------------------------------------------
// Each layout gives HDR (header slots at the line start), DATA (bases per line), MID (slot 256, the
// 64-byte half boundary), WORDS (packed input words per line), the offset-array geometry
// (SB_LINES, SB_LOG, SHIFT, Super), the exact division by DATA (MAGIC, MAGIC_T; and LINE32_SHIFT,
// LINE32_MAGIC for 32-bit positions), and
//   MULTI    false: a query counts between its slot p and the middle (within p's 64-byte half);
//            true:  between p and the nearest of three anchors, within p's 64-slot pair (24_8);
//   offset1(s, j, c) / offset4 + delta(a, b, c, p, j) = rank(anchor of p, c), where a and b hold the
//            line's first eight u32 words (the header) and p is the query's line slot.
// The arithmetic is modulo 2^64: a paired layout's offset may exceed the anchor rank (its delta
// carries a negative bias), and the sum is still exact.
//
// QR16: four 16-bit deltas in slots [0,32) (lo_0 low half = A | C << 16, hi_0 low half = G | T << 16),
//       480 bases, 128 lines per superblock, offsets s = floor(rank / 2^12) as u32.
// QR32: four 32-bit deltas in slots [0,64) (lo_0 = A | C << 32, hi_0 = G | T << 32), 448 bases,
//       2^23 lines per superblock, exact u64 offsets.  floor(x/448) = mulhi(x, ceil(2^72/448)) >> 8,
//       exact for x < 2^63 (e = 384 < 448).
struct QR16 {
    static constexpr int ID = QR_LAYOUT_16;
    static constexpr uint32_t HDR = 32, DATA = 480, MID = 256, WORDS = 15;
    static constexpr bool MULTI = false;
    static constexpr uint64_t SB_LINES = 128;
    static constexpr uint32_t SB_LOG = 7, SHIFT = 12;
    static constexpr uint64_t MAGIC = QR_MAGIC;
    static constexpr uint32_t MAGIC_T = QR_MAGIC_T;
    static constexpr uint32_t LINE32_SHIFT = 5, LINE32_MAGIC = 0x11111112u;  // 480 = 2^5 * 15
    static constexpr uint64_t MAX_N = (1ull << 44) - 1;
    using Super = uint32_t;
    __device__ __forceinline__ static uint64_t delta(const uint4 &a, const uint4 &, uint32_t c, uint32_t, uint64_t) {
        const uint32_t m2 = 0u - ((c >> 1) & 1u);
        const uint32_t d = (a.x & ~m2) | (a.z & m2);
        return (d >> (16u * (c & 1u))) & 0xffffu;
    }
    __device__ __forceinline__ static uint64_t offset1(const Super *__restrict__ s, uint64_t j, uint32_t c) {
        return (uint64_t)sel4(reinterpret_cast<const uint4 *>(s)[j >> SB_LOG], c) << SHIFT;
    }
    __device__ __forceinline__ static void offset4(const Super *__restrict__ s, uint64_t j, uint64_t (&o)[4]) {
        const uint4 v = reinterpret_cast<const uint4 *>(s)[j >> SB_LOG];
        o[0] = (uint64_t)v.x << SHIFT, o[1] = (uint64_t)v.y << SHIFT, o[2] = (uint64_t)v.z << SHIFT,
        o[3] = (uint64_t)v.w << SHIFT;
    }
};

// QR16 with paired superblocks (the paper's appendix on pairing superblocks): one row of four
// shifted offsets per 256 lines, taken at the pair's middle (line 128 of the 256), so half the
// offsets of QR16.  Lines of the lower 128 store their delta plus BIAS = 128 * 480 - 224 (the most
// bases between a lower line's middle and the pair's middle), removed again by the query.
//   b_{j,c} = rank(480 j + 224, c) - 2^12 s'_{j/256, c} + [j mod 256 < 128] BIAS
//   s'_{i,c} = floor(rank(480 (256 i + 128), c) / 2^12)
//   bounds: lower lines 0 <= b <= BIAS + 4095 = 65311; upper lines b <= 127*480 + 224 + 4095 = 65279
struct QR16P {
    static constexpr int ID = QR_LAYOUT_16P;
    static constexpr uint32_t HDR = 32, DATA = 480, MID = 256, WORDS = 15;
    static constexpr bool MULTI = false;
    static constexpr uint64_t SB_LINES = 256;
    static constexpr uint32_t SB_LOG = 8, SHIFT = 12;
    static constexpr uint64_t BIAS = 128 * 480 - 224;
    static constexpr uint64_t MAGIC = QR_MAGIC;
    static constexpr uint32_t MAGIC_T = QR_MAGIC_T;
    static constexpr uint32_t LINE32_SHIFT = QR16::LINE32_SHIFT, LINE32_MAGIC = QR16::LINE32_MAGIC;
    static constexpr uint64_t MAX_N = (1ull << 44) - 1;
    using Super = uint32_t;
    __device__ __forceinline__ static uint64_t delta(const uint4 &a, const uint4 &b, uint32_t c, uint32_t p, uint64_t j) {
        return QR16::delta(a, b, c, p, j) - ((j & 128u) ? 0ull : BIAS);
    }
    __device__ __forceinline__ static uint64_t offset1(const Super *__restrict__ s, uint64_t j, uint32_t c) {
        return (uint64_t)sel4(reinterpret_cast<const uint4 *>(s)[j >> SB_LOG], c) << SHIFT;
    }
    __device__ __forceinline__ static void offset4(const Super *__restrict__ s, uint64_t j, uint64_t (&o)[4]) {
        const uint4 v = reinterpret_cast<const uint4 *>(s)[j >> SB_LOG];
        o[0] = (uint64_t)v.x << SHIFT, o[1] = (uint64_t)v.y << SHIFT, o[2] = (uint64_t)v.z << SHIFT,
        o[3] = (uint64_t)v.w << SHIFT;
    }
};

struct QR32 {
    static constexpr int ID = QR_LAYOUT_32;
    static constexpr uint32_t HDR = 64, DATA = 448, MID = 256, WORDS = 14;
    static constexpr bool MULTI = false;
    static constexpr uint64_t SB_LINES = 1ull << 23;
    static constexpr uint32_t SB_LOG = 23, SHIFT = 0;
    static constexpr uint64_t MAGIC = 0x924924924924924aull;  // ceil(2^72 / 448)
    static constexpr uint32_t MAGIC_T = 8;
    static constexpr uint32_t LINE32_SHIFT = 6, LINE32_MAGIC = 0x24924925u;  // 448 = 2^6 * 7
    static constexpr uint64_t MAX_N = (1ull << 48) - 1;
    using Super = uint64_t;
    __device__ __forceinline__ static uint64_t delta(const uint4 &a, const uint4 &, uint32_t c, uint32_t, uint64_t) {
        return sel4(a, c);
    }
    __device__ __forceinline__ static uint64_t offset1(const Super *__restrict__ s, uint64_t j, uint32_t c) {
        return s[4 * (j >> SB_LOG) + (c & 3u)];
    }
    __device__ __forceinline__ static void offset4(const Super *__restrict__ s, uint64_t j, uint64_t (&o)[4]) {
        const ulonglong2 *p = reinterpret_cast<const ulonglong2 *>(s + 4 * (j >> SB_LOG));
        const ulonglong2 a = p[0], b = p[1];
        o[0] = a.x, o[1] = a.y, o[2] = b.x, o[3] = b.y;
    }
};

// 64-bit word x of the header (u32 words 2x, 2x+1 of a.xyzw, b.xyzw) for a runtime x in 0..3.
__device__ __forceinline__ uint64_t hdr64(const uint4 &a, const uint4 &b, uint32_t x) {
    const uint32_t m1 = 0u - (x & 1u), m2 = 0u - ((x >> 1) & 1u);
    const uint32_t lo = (((a.x & ~m1) | (a.z & m1)) & ~m2) | (((b.x & ~m1) | (b.z & m1)) & m2);
    const uint32_t hi = (((a.y & ~m1) | (a.w & m1)) & ~m2) | (((b.y & ~m1) | (b.w & m1)) & m2);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

// The paper's QuadRank64: the line's first two pairs (slots [0,128), u64 words 0..3) hold the
// absolute ranks of A, C, G, T at the line's middle (slot 256 = data base 128), then 384 bases in
// pairs 2..7; no offset array.  floor(x/384) = mulhi(x, ceil(2^72/384)) >> 8, exact for x < 2^63
// (e = 128 < 384).
struct QR64 {
    static constexpr int ID = QR_LAYOUT_64;
    static constexpr uint32_t HDR = 128, DATA = 384, MID = 256, WORDS = 12;
    static constexpr bool MULTI = false;
    static constexpr uint64_t SB_LINES = 0;  // no offset array
    static constexpr uint32_t SB_LOG = 0, SHIFT = 0;
    static constexpr uint64_t MAGIC = 0xaaaaaaaaaaaaaaabull;  // ceil(2^72 / 384)
    static constexpr uint32_t MAGIC_T = 8;
    static constexpr uint32_t LINE32_SHIFT = 7, LINE32_MAGIC = 0x55555556u;  // 384 = 2^7 * 3
    static constexpr uint64_t MAX_N = (1ull << 48) - 1;
    using Super = uint64_t;
    __device__ __forceinline__ static uint64_t delta(const uint4 &a, const uint4 &b, uint32_t c, uint32_t, uint64_t) {
        return hdr64(a, b, c);
    }
    __device__ __forceinline__ static uint64_t offset1(const Super *__restrict__, uint64_t, uint32_t) { return 0; }
    __device__ __forceinline__ static void offset4(const Super *__restrict__, uint64_t, uint64_t (&o)[4]) {
        o[0] = o[1] = o[2] = o[3] = 0;
    }
};

// The paper's QuadRank24_8 on 128-byte lines: the header (slots [0,128)) holds per symbol a 24-bit
// delta L1 to the anchor at slot 192 and two 8-bit deltas d1 (from slot 192 to 320) and d2 (from 320
// to 448); 384 bases fill pairs 2..7, and a query counts at most one 64-slot pair, backwards to the
// anchor at its end (pairs 2, 4, 6) or forwards from the anchor at its start (pairs 3, 5, 7).
//   u32 word c (c = A..T): L1_c | d1_c << 24;  u32 word 4 + c: d2_c
//   L1_{j,c} = rank(384 j + 64, c) - S_{j/2^15, c};  d1 = #c in bases [64, 192) of the line, d2 in
//   [192, 320) (each <= 128);  S exact (u64) per 2^15 lines;  L1 <= (2^15 - 1)*384 + 64 < 2^24
struct QR24_8 {
    static constexpr int ID = QR_LAYOUT_24_8;
    static constexpr uint32_t HDR = 128, DATA = 384, MID = 256, WORDS = 12;
    static constexpr bool MULTI = true;
    static constexpr uint64_t SB_LINES = 1ull << 15;
    static constexpr uint32_t SB_LOG = 15, SHIFT = 0;
    static constexpr uint64_t MAGIC = QR64::MAGIC;
    static constexpr uint32_t MAGIC_T = QR64::MAGIC_T;
    static constexpr uint32_t LINE32_SHIFT = QR64::LINE32_SHIFT, LINE32_MAGIC = QR64::LINE32_MAGIC;
    static constexpr uint64_t MAX_N = (1ull << 48) - 1;
    using Super = uint64_t;
    __device__ __forceinline__ static uint64_t delta(const uint4 &a, const uint4 &b, uint32_t c, uint32_t p, uint64_t) {
        const uint32_t w = sel4(a, c), d2 = sel4(b, c) & 0xffu;
        return (uint64_t)(w & 0xffffffu) + (p >= 256 ? (w >> 24) : 0u) + (p >= 384 ? d2 : 0u);
    }
    __device__ __forceinline__ static uint64_t offset1(const Super *__restrict__ s, uint64_t j, uint32_t c) {
        return s[4 * (j >> SB_LOG) + (c & 3u)];
    }
    __device__ __forceinline__ static void offset4(const Super *__restrict__ s, uint64_t j, uint64_t (&o)[4]) {
        const ulonglong2 *p = reinterpret_cast<const ulonglong2 *>(s + 4 * (j >> SB_LOG));
        const ulonglong2 a = p[0], b = p[1];
        o[0] = a.x, o[1] = a.y, o[2] = b.x, o[3] = b.y;
    }
};

template <class L>
__host__ __device__ __forceinline__ uint64_t qline_of(uint64_t q) {
    return mulhi64(q, L::MAGIC) >> L::MAGIC_T;
}

// floor(q / DATA) for every 32-bit q with one 32-bit multiply-high.  DATA = 2^s d with d odd
// (480 = 2^5 * 15, 448 = 2^6 * 7, 384 = 2^7 * 3) and m = ceil(2^32 / d) has e = m d - 2^32 = 14, 3
// and 2, so floor(y m / 2^32) = floor(y / d) wherever y e < 2^32, which covers y = q >> s < 2^27.
// (Checked against division for all 2^32 values of q.)
template <class L>
__host__ __device__ __forceinline__ uint32_t qline_of32(uint32_t q) {
    return (uint32_t)(((uint64_t)(q >> L::LINE32_SHIFT) * L::LINE32_MAGIC) >> 32);
}

// ---- lane-pair form: lane hf (0/1) of a pair holds half hf of the line -------------------------
struct PairHalf {
    uint32_t w[16];  // half hf of the line, same word order as HalfLine::w
    uint32_t t;      // slot of q inside the half that contains it
    bool up;         // q lies in the upper half
    uint64_t j;      // line index
};

template <class L>
__device__ __forceinline__ void load_pair_half(const uint4 *__restrict__ lines, uint64_t q, uint32_t hf, PairHalf &ph) {
    ph.j = qline_of<L>(q);
    const uint32_t p = (uint32_t)(q - ph.j * L::DATA) + L::HDR;
    ph.up = p >= L::MID;
    ph.t = ph.up ? p - L::MID : p;
    const uint4 *H = lines + ph.j * 8 + hf * 4;
    const uint4 a = H[0], b = H[1], c = H[2], d = H[3];
    ph.w[0] = a.x, ph.w[1] = a.y, ph.w[2] = a.z, ph.w[3] = a.w;
    ph.w[4] = b.x, ph.w[5] = b.y, ph.w[6] = b.z, ph.w[7] = b.w;
    ph.w[8] = c.x, ph.w[9] = c.y, ph.w[10] = c.z, ph.w[11] = c.w;
    ph.w[12] = d.x, ph.w[13] = d.y, ph.w[14] = d.z, ph.w[15] = d.w;
}

// Occurrences of c in this lane's share of the counted range (zero unless the lane holds q's half).
__device__ __forceinline__ uint32_t pair_count1(const PairHalf &ph, uint32_t hf, uint32_t c) {
    if ((uint32_t)ph.up != hf) return 0u;
    const uint32_t inv = ph.up ? 0u : 0xffffffffu;
    const uint32_t xl = (c & 1) ? 0u : 0xffffffffu, xh = (c & 2) ? 0u : 0xffffffffu;
    uint32_t cnt = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
#pragma unroll
        for (int sub = 0; sub < 2; ++sub) {
            const uint32_t m = prefix_mask32(ph.t, 2 * k + sub) ^ inv;
            cnt += __popc((ph.w[4 * k + sub] ^ xl) & (ph.w[4 * k + 2 + sub] ^ xh) & m);
        }
    }
    return cnt;
}

// Slots of this lane's share of the range whose symbol is at most c (zero unless the lane holds q's
// half).  Symbol s = lo + 2 hi exceeds c exactly where: c = A: lo | hi; c = C: hi; c = G: lo & hi;
// c = T: nowhere.  Counted as the range length minus the slots above c.
__device__ __forceinline__ uint32_t pair_count_le(const PairHalf &ph, uint32_t hf, uint32_t c) {
    if ((uint32_t)ph.up != hf) return 0u;
    const uint32_t inv = ph.up ? 0u : 0xffffffffu;
    const uint32_t ma = 0u - (c & 1u), mb = 0u - ((c >> 1) & 1u);
    uint32_t gt = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
#pragma unroll
        for (int sub = 0; sub < 2; ++sub) {
            const uint32_t m = prefix_mask32(ph.t, 2 * k + sub) ^ inv;
            const uint32_t lo = ph.w[4 * k + sub], hi = ph.w[4 * k + 2 + sub];
            const uint32_t above = (mb & lo & hi & ~ma) | (~mb & (hi | (lo & ~ma)));
            gt += __popc(above & m);
        }
    }
    return (ph.up ? ph.t : QR_MID - ph.t) - gt;
}

// Sums over the symbols x <= c of the line deltas and of the superblock offsets.
template <class L>
__device__ __forceinline__ uint64_t delta_le(const uint4 &a, const uint4 &b, uint32_t c, uint32_t p, uint64_t j) {
    uint64_t d = 0;
#pragma unroll
    for (uint32_t x = 0; x < 4; ++x) d += x <= c ? L::delta(a, b, x, p, j) : 0ull;
    return d;
}

// The header words (line u32 words 0..7) of a lane pair's lower half.
__device__ __forceinline__ uint4 hdr_lo(const uint32_t (&w)[16]) { return make_uint4(w[0], w[1], w[2], w[3]); }
__device__ __forceinline__ uint4 hdr_hi(const uint32_t (&w)[16]) { return make_uint4(w[4], w[5], w[6], w[7]); }

template <class L>
__device__ __forceinline__ uint64_t offset_le(const typename L::Super *__restrict__ s, uint64_t j, uint32_t c) {
    if constexpr (L::SB_LINES == 0) return 0;  // no offset array
    uint64_t o[4];
    L::offset4(s, j, o);
    return o[0] + (c >= 1 ? o[1] : 0ull) + (c >= 2 ? o[2] : 0ull) + (c >= 3 ? o[3] : 0ull);
}

__device__ __forceinline__ void pair_count4(const PairHalf &ph, uint32_t hf, uint32_t (&cnt)[4]) {
    if ((uint32_t)ph.up != hf) {
        cnt[0] = cnt[1] = cnt[2] = cnt[3] = 0u;
        return;
    }
    const uint32_t inv = ph.up ? 0u : 0xffffffffu;
    uint32_t cT = 0, cL = 0, cH = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
#pragma unroll
        for (int sub = 0; sub < 2; ++sub) {
            const uint32_t m = prefix_mask32(ph.t, 2 * k + sub) ^ inv;
            const uint32_t lo = ph.w[4 * k + sub] & m, hi = ph.w[4 * k + 2 + sub] & m;
            cT += __popc(lo & hi);
            cL += __popc(lo);
            cH += __popc(hi);
        }
    }
    const uint32_t len = ph.up ? ph.t : QR_MID - ph.t;
    cnt[0] = len - cL - cH + cT;
    cnt[1] = cL - cT;
    cnt[2] = cH - cT;
    cnt[3] = cT;
}

// ---- counts of any layout ------------------------------------------------------------------------
// The four words (lo low, lo high, hi low, hi high) of pair k (0..3) of a half line, picked with
// masks.
__device__ __forceinline__ void pick_pair(const uint32_t (&w)[16], uint32_t k, uint32_t (&o)[4]) {
    o[0] = o[1] = o[2] = o[3] = 0u;
#pragma unroll
    for (uint32_t s = 0; s < 4; ++s) {
        const uint32_t m = (k == s) ? 0xffffffffu : 0u;
        o[0] |= w[4 * s] & m, o[1] |= w[4 * s + 1] & m, o[2] |= w[4 * s + 2] & m, o[3] |= w[4 * s + 3] & m;
    }
}

// The counted range of a multi-anchor layout: pair k = t / 64 of q's half, slots [u, 64) of it
// before an anchor (k even) or [0, u) after one (k odd), u = t mod 64.  Masks of its two 32-slot
// words, and whether the range follows its anchor.
__device__ __forceinline__ bool multi_masks(uint32_t t, uint32_t &m0, uint32_t &m1) {
    const bool fwd = (t >> 6) & 1u;
    const uint32_t u = t & 63u, inv = fwd ? 0u : 0xffffffffu;
    m0 = prefix_mask32(u, 0) ^ inv;
    m1 = prefix_mask32(u, 1) ^ inv;
    return fwd;
}

// Occurrences of c in this lane's share of the counted range (zero unless the lane holds q's half),
// and whether the range follows the anchor (add) or precedes it (subtract).
template <class L>
__device__ __forceinline__ uint32_t count1(const PairHalf &ph, uint32_t hf, uint32_t c, bool &fwd) {
    if constexpr (L::MULTI) {
        uint32_t m0, m1, v[4];
        fwd = multi_masks(ph.t, m0, m1);
        if ((uint32_t)ph.up != hf) return 0u;
        pick_pair(ph.w, ph.t >> 6, v);
        const uint32_t xl = (c & 1) ? 0u : 0xffffffffu, xh = (c & 2) ? 0u : 0xffffffffu;
        return __popc((v[0] ^ xl) & (v[2] ^ xh) & m0) + __popc((v[1] ^ xl) & (v[3] ^ xh) & m1);
    } else {
        fwd = ph.up;
        return pair_count1(ph, hf, c);
    }
}

// Slots of the counted range whose symbol is at most c (see pair_count_le).
template <class L>
__device__ __forceinline__ uint32_t count_le(const PairHalf &ph, uint32_t hf, uint32_t c, bool &fwd) {
    if constexpr (L::MULTI) {
        uint32_t m0, m1, v[4];
        fwd = multi_masks(ph.t, m0, m1);
        if ((uint32_t)ph.up != hf) return 0u;
        pick_pair(ph.w, ph.t >> 6, v);
        const uint32_t ma = 0u - (c & 1u), mb = 0u - ((c >> 1) & 1u);
        const uint32_t a0 = (mb & v[0] & v[2] & ~ma) | (~mb & (v[2] | (v[0] & ~ma)));
        const uint32_t a1 = (mb & v[1] & v[3] & ~ma) | (~mb & (v[3] | (v[1] & ~ma)));
        const uint32_t len = fwd ? (ph.t & 63u) : 64u - (ph.t & 63u);
        return len - __popc(a0 & m0) - __popc(a1 & m1);
    } else {
        fwd = ph.up;
        return pair_count_le(ph, hf, c);
    }
}

// The four symbol counts of the counted range (zero unless the lane holds q's half).
template <class L>
__device__ __forceinline__ void count4(const PairHalf &ph, uint32_t hf, uint32_t (&cnt)[4], bool &fwd) {
    if constexpr (L::MULTI) {
        uint32_t m0, m1, v[4];
        fwd = multi_masks(ph.t, m0, m1);
        if ((uint32_t)ph.up != hf) {
            cnt[0] = cnt[1] = cnt[2] = cnt[3] = 0u;
            return;
        }
        pick_pair(ph.w, ph.t >> 6, v);
        const uint32_t l0 = v[0] & m0, l1 = v[1] & m1, h0 = v[2] & m0, h1 = v[3] & m1;
        const uint32_t cT = __popc(l0 & h0) + __popc(l1 & h1), cL = __popc(l0) + __popc(l1),
                       cH = __popc(h0) + __popc(h1);
        const uint32_t len = fwd ? (ph.t & 63u) : 64u - (ph.t & 63u);
        cnt[0] = len - cL - cH + cT;
        cnt[1] = cL - cT;
        cnt[2] = cH - cT;
        cnt[3] = cT;
    } else {
        fwd = ph.up;
        pair_count4(ph, hf, cnt);
    }
}

// ---- one lane per query, 32-bit positions (the FM-index search) ---------------------------------
// Every rank of an FM-index is below 2^32 (its BWT has fewer than 2^32 rows), so the offsets and
// deltas are summed modulo 2^32: the low words of the 64-bit sums, hence exact.

// The 64-byte half line that holds a position, read by one lane, with the line's header (its first
// 32 bytes, which hold the deltas of every layout) and its offsets.
struct LaneHalf {
    uint32_t w[16];  // the half: pair k (0..3) = lo_k (w[4k], w[4k+1]), hi_k (w[4k+2], w[4k+3])
    uint4 h0, h1;    // line bytes [0, 16) and [16, 32)
    uint32_t off[4]; // offsets of A, C, G, T (low 32 bits)
    uint32_t j;      // line index
};

// Slot of position q in its line (header slots first).
template <class L>
__device__ __forceinline__ uint32_t lane_slot(uint32_t q, uint32_t j) {
    return q - j * L::DATA + L::HDR;
}

// Load the half line of q.  For q in the upper half the header words are loaded on their own (the
// second 16 bytes only where the layout's header is wider than 64 slots); in the lower half they
// are the half's first words.
template <class L>
__device__ __forceinline__ void load_lane_half(const uint4 *__restrict__ lines, const typename L::Super *__restrict__ super,
                                               uint32_t q, LaneHalf &hl) {
    hl.j = qline_of32<L>(q);
    const bool up = lane_slot<L>(q, hl.j) >= L::MID;
    const uint4 *Ln = lines + (uint64_t)hl.j * 8;
    const uint4 *H = Ln + (up ? 4 : 0);
    const uint4 a = H[0], b = H[1], c = H[2], d = H[3];
    hl.w[0] = a.x, hl.w[1] = a.y, hl.w[2] = a.z, hl.w[3] = a.w;
    hl.w[4] = b.x, hl.w[5] = b.y, hl.w[6] = b.z, hl.w[7] = b.w;
    hl.w[8] = c.x, hl.w[9] = c.y, hl.w[10] = c.z, hl.w[11] = c.w;
    hl.w[12] = d.x, hl.w[13] = d.y, hl.w[14] = d.z, hl.w[15] = d.w;
    if (up) {
        hl.h0 = Ln[0];
        if constexpr (L::HDR > 64) hl.h1 = Ln[1];
        else hl.h1 = make_uint4(0u, 0u, 0u, 0u);
    } else {
        hl.h0 = a;
        hl.h1 = b;
    }
    if constexpr (L::SB_LINES == 0) {
        hl.off[0] = hl.off[1] = hl.off[2] = hl.off[3] = 0u;
    } else {
        uint64_t o[4];
        L::offset4(super, hl.j, o);
        hl.off[0] = (uint32_t)o[0], hl.off[1] = (uint32_t)o[1], hl.off[2] = (uint32_t)o[2], hl.off[3] = (uint32_t)o[3];
    }
}

// rank(q, c) (modulo 2^32) for a position q whose half line hl holds, given q's line slot p.  The
// count runs from p to the half's boundary with the middle, or (multi-anchor layouts) to the nearest
// anchor within p's 64-slot pair.
template <class L>
__device__ __forceinline__ uint32_t lane_rank(const LaneHalf &hl, uint32_t p, uint32_t c) {
    const bool up = p >= L::MID;
    const uint32_t t = up ? p - L::MID : p;
    const uint32_t anchor =
        sel4(make_uint4(hl.off[0], hl.off[1], hl.off[2], hl.off[3]), c) + (uint32_t)L::delta(hl.h0, hl.h1, c, p, hl.j);
    const uint32_t xl = (c & 1) ? 0u : 0xffffffffu, xh = (c & 2) ? 0u : 0xffffffffu;
    bool fwd;
    uint32_t cnt = 0;
    if constexpr (L::MULTI) {
        uint32_t m0, m1, v[4];
        fwd = multi_masks(t, m0, m1);
        pick_pair(hl.w, t >> 6, v);
        cnt = __popc((v[0] ^ xl) & (v[2] ^ xh) & m0) + __popc((v[1] ^ xl) & (v[3] ^ xh) & m1);
    } else {
        fwd = up;
        const uint32_t inv = up ? 0u : 0xffffffffu;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
#pragma unroll
            for (int sub = 0; sub < 2; ++sub) {
                const uint32_t m = prefix_mask32(t, 2 * k + sub) ^ inv;
                cnt += __popc((hl.w[4 * k + sub] ^ xl) & (hl.w[4 * k + 2 + sub] ^ xh) & m);
            }
        }
    }
    return fwd ? anchor + cnt : anchor - cnt;
}

// The symbol at line slot p of the half line hl, picked with masks.
__device__ __forceinline__ uint32_t lane_symbol(const LaneHalf &hl, uint32_t p) {
    const uint32_t t = p & 255u;
    const uint32_t word = t >> 5;  // 32-slot word of the half: pair word >> 1, its low/high u32 word & 1
    uint32_t lo = 0, hi = 0;
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
#pragma unroll
        for (uint32_t sub = 0; sub < 2; ++sub) {
            const uint32_t m = (word == 2 * k + sub) ? 0xffffffffu : 0u;
            lo |= hl.w[4 * k + sub] & m;
            hi |= hl.w[4 * k + 2 + sub] & m;
        }
    }
    const uint32_t b = t & 31u;
    return ((lo >> b) & 1u) | (((hi >> b) & 1u) << 1);
}

}  // namespace qr
