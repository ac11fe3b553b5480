// Device-side QuadRank query primitives (layout described in quadrank.hip), shared by the rank
// kernels and the FM-index search.
#pragma once

#include "common.hpp"

namespace qr {

// The half line that holds query position q, plus what is needed to finish rank(q, .).
struct HalfLine {
    uint32_t w[16];  // the 64-byte half: pair k (0..3) = lo_k (w[4k], w[4k+1]), hi_k (w[4k+2], w[4k+3])
    uint32_t dAC;    // b_A | b_C << 16
    uint32_t dGT;    // b_G | b_T << 16
    uint4 s;         // the four superblock offsets s_{i,A..T}
    uint32_t t;      // slot of q inside the half (0..255)
    bool up;         // q lies in the upper half (count forward from the middle)
};

__device__ __forceinline__ void load_half(const uint4 *__restrict__ lines, const uint32_t *__restrict__ super,
                                          uint64_t q, HalfLine &hl) {
    const uint64_t j = qr_line_of(q);
    const uint32_t p = (uint32_t)(q - j * QR_DATA_BASES) + QR_HDR;
    hl.up = p >= QR_MID;
    hl.t = hl.up ? p - QR_MID : p;
    const uint4 *L = lines + j * 8;
    const uint4 *H = L + (hl.up ? 4 : 0);
    const uint4 a = H[0], b = H[1], c = H[2], d = H[3];
    hl.w[0] = a.x, hl.w[1] = a.y, hl.w[2] = a.z, hl.w[3] = a.w;
    hl.w[4] = b.x, hl.w[5] = b.y, hl.w[6] = b.z, hl.w[7] = b.w;
    hl.w[8] = c.x, hl.w[9] = c.y, hl.w[10] = c.z, hl.w[11] = c.w;
    hl.w[12] = d.x, hl.w[13] = d.y, hl.w[14] = d.z, hl.w[15] = d.w;
    if (hl.up) {
        const uint4 h0 = L[0];
        hl.dAC = h0.x, hl.dGT = h0.z;
    } else {
        hl.dAC = a.x, hl.dGT = a.z;
    }
    hl.s = reinterpret_cast<const uint4 *>(super)[j / QR_LINES_PER_SB];
}

// load_half for positions below 2^32 (every position of an FM-index, whose BWT has fewer than 2^32
// rows), with 32-bit line arithmetic.
__device__ __forceinline__ void load_half32(const uint4 *__restrict__ lines, const uint32_t *__restrict__ super,
                                            uint32_t q, HalfLine &hl) {
    const uint32_t j = qr_line_of32(q);
    const uint32_t p = q - j * (uint32_t)QR_DATA_BASES + QR_HDR;
    hl.up = p >= QR_MID;
    hl.t = hl.up ? p - QR_MID : p;
    const uint4 *L = lines + (uint64_t)j * 8;
    const uint4 *H = L + (hl.up ? 4 : 0);
    const uint4 a = H[0], b = H[1], c = H[2], d = H[3];
    hl.w[0] = a.x, hl.w[1] = a.y, hl.w[2] = a.z, hl.w[3] = a.w;
    hl.w[4] = b.x, hl.w[5] = b.y, hl.w[6] = b.z, hl.w[7] = b.w;
    hl.w[8] = c.x, hl.w[9] = c.y, hl.w[10] = c.z, hl.w[11] = c.w;
    hl.w[12] = d.x, hl.w[13] = d.y, hl.w[14] = d.z, hl.w[15] = d.w;
    if (hl.up) {
        const uint4 h0 = L[0];
        hl.dAC = h0.x, hl.dGT = h0.z;
    } else {
        hl.dAC = a.x, hl.dGT = a.z;
    }
    hl.s = reinterpret_cast<const uint4 *>(super)[j / QR_LINES_PER_SB];
}

// v.{x,y,z,w}[c] by mask arithmetic: a runtime-indexed select chain would be lowered to a
// stack array (scratch memory) once several queries are unrolled per lane.
__device__ __forceinline__ uint32_t sel4(const uint4 &v, uint32_t c) {
    const uint32_t m1 = 0u - (c & 1u), m2 = 0u - ((c >> 1) & 1u);
    const uint32_t lo = (v.x & ~m1) | (v.y & m1), hi = (v.z & ~m1) | (v.w & m1);
    return (lo & ~m2) | (hi & m2);
}

__device__ __forceinline__ uint32_t delta_of(const HalfLine &hl, uint32_t c) {
    const uint32_t m2 = 0u - ((c >> 1) & 1u);
    const uint32_t d = (hl.dAC & ~m2) | (hl.dGT & m2);
    return (d >> (16u * (c & 1u))) & 0xffffu;
}

// Occurrences of c in the counted range of the half: slots [0, t) if up, else [t, 256).
__device__ __forceinline__ uint32_t half_count1(const HalfLine &hl, uint32_t c) {
    const uint32_t inv = hl.up ? 0u : 0xffffffffu;
    const uint32_t xl = (c & 1) ? 0u : 0xffffffffu, xh = (c & 2) ? 0u : 0xffffffffu;
    uint32_t cnt = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
#pragma unroll
        for (int sub = 0; sub < 2; ++sub) {
            const uint32_t lo = hl.w[4 * k + sub], hi = hl.w[4 * k + 2 + sub];
            const uint32_t m = prefix_mask32(hl.t, 2 * k + sub) ^ inv;
            cnt += __popc((lo ^ xl) & (hi ^ xh) & m);
        }
    }
    return cnt;
}

__device__ __forceinline__ uint64_t rank1_from_half(const HalfLine &hl, uint32_t c) {
    const uint64_t mid = ((uint64_t)sel4(hl.s, c) << QR_SHIFT) + delta_of(hl, c);
    const uint32_t cnt = half_count1(hl, c);
    return hl.up ? mid + cnt : mid - cnt;
}

// rank1_from_half in 32-bit arithmetic, for structures whose every rank is below 2^32 (then the
// shifted offset, the mid-line rank and the result all fit).
__device__ __forceinline__ uint32_t rank1_from_half32(const HalfLine &hl, uint32_t c) {
    const uint32_t mid = (sel4(hl.s, c) << QR_SHIFT) + delta_of(hl, c);
    const uint32_t cnt = half_count1(hl, c);
    return hl.up ? mid + cnt : mid - cnt;
}

// The symbol stored at the slot of q (the half line's slot t), picked with masks.
__device__ __forceinline__ uint32_t symbol_from_half(const HalfLine &hl) {
    const uint32_t word = hl.t >> 5;  // 32-slot word of the half: pair word >> 1, its low/high u32 word & 1
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
    const uint32_t b = hl.t & 31u;
    return ((lo >> b) & 1u) | (((hi >> b) & 1u) << 1);
}

__device__ __forceinline__ void rank4_from_half(const HalfLine &hl, uint64_t (&r)[4]) {
    const uint32_t inv = hl.up ? 0u : 0xffffffffu;
    uint32_t cT = 0, cL = 0, cH = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
#pragma unroll
        for (int sub = 0; sub < 2; ++sub) {
            const uint32_t m = prefix_mask32(hl.t, 2 * k + sub) ^ inv;
            const uint32_t lo = hl.w[4 * k + sub] & m, hi = hl.w[4 * k + 2 + sub] & m;
            cT += __popc(lo & hi);
            cL += __popc(lo);
            cH += __popc(hi);
        }
    }
    const uint32_t len = hl.up ? hl.t : QR_MID - hl.t;
    const uint32_t cnt[4] = {len - cL - cH + cT, cL - cT, cH - cT, cT};
#pragma unroll
    for (uint32_t c = 0; c < 4; ++c) {
        const uint64_t mid = ((uint64_t)sel4(hl.s, c) << QR_SHIFT) + delta_of(hl, c);
        r[c] = hl.up ? mid + cnt[c] : mid - cnt[c];
    }
}

// ---- layouts -------------------------------------------------------------------------------------
// QR16: four 16-bit deltas in slots [0,32) (lo_0 low half = A | C << 16, hi_0 low half = G | T << 16),
//       480 bases, 128 lines per superblock, offsets s = floor(rank / 2^12) as u32.
// QR32: four 32-bit deltas in slots [0,64) (lo_0 = A | C << 32, hi_0 = G | T << 32), 448 bases,
//       2^23 lines per superblock, exact u64 offsets.  floor(x/448) = mulhi(x, ceil(2^72/448)) >> 8,
//       exact for x < 2^63 (e = 384 < 448).
struct QR16 {
    static constexpr uint32_t HDR = 32, DATA = 480, MID = 256, WORDS = 15;
    static constexpr uint64_t SB_LINES = 128;
    static constexpr uint32_t SB_LOG = 7, SHIFT = 12;
    static constexpr uint64_t MAGIC = QR_MAGIC;
    static constexpr uint32_t MAGIC_T = QR_MAGIC_T;
    static constexpr uint64_t MAX_N = (1ull << 44) - 1;
    using Super = uint32_t;
    // delta of symbol c from the line's first four u32 words
    __device__ __forceinline__ static uint32_t delta(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3, uint32_t c) {
        (void)w1, (void)w3;
        const uint32_t m2 = 0u - ((c >> 1) & 1u);
        const uint32_t d = (w0 & ~m2) | (w2 & m2);
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

struct QR32 {
    static constexpr uint32_t HDR = 64, DATA = 448, MID = 256, WORDS = 14;
    static constexpr uint64_t SB_LINES = 1ull << 23;
    static constexpr uint32_t SB_LOG = 23, SHIFT = 0;
    static constexpr uint64_t MAGIC = 0x924924924924924aull;  // ceil(2^72 / 448)
    static constexpr uint32_t MAGIC_T = 8;
    static constexpr uint64_t MAX_N = (1ull << 48) - 1;
    using Super = uint64_t;
    __device__ __forceinline__ static uint32_t delta(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3, uint32_t c) {
        const uint32_t m1 = 0u - (c & 1u), m2 = 0u - ((c >> 1) & 1u);
        const uint32_t lo = (w0 & ~m1) | (w1 & m1), hi = (w2 & ~m1) | (w3 & m1);
        return (lo & ~m2) | (hi & m2);
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
__device__ __forceinline__ uint64_t delta_le(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3, uint32_t c) {
    uint64_t d = 0;
#pragma unroll
    for (uint32_t x = 0; x < 4; ++x) d += x <= c ? (uint64_t)L::delta(w0, w1, w2, w3, x) : 0ull;
    return d;
}

template <class L>
__device__ __forceinline__ uint64_t offset_le(const typename L::Super *__restrict__ s, uint64_t j, uint32_t c) {
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

}  // namespace qr
