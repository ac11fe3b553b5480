// Device-side BiRank layout traits and a one-lane rank, shared by the BiRank kernels and by the
// FM-index's locate walk (which ranks over the bitvector of sampled suffix-array rows).  The layouts
// are described with the BiRank kernels.
#pragma once

#include "common.hpp"

namespace qr {

// Every layout is described by: HDR (header bits at the line start), DATA (input bits per line), MID
// (line bit 512, the 64-byte half boundary), the offset-array geometry (SB_LINES lines per entry,
// SHIFT, Super), the exact division by DATA (MAGIC, MAGIC_T), and
//   QUARTER  false: a query counts from the line's middle to q (within q's 64-byte half);
//            true:  from the middle of q's half (line bit 256 or 768) to q (within a quarter line);
//   offset(s, j) + delta(w0, w1, up, j) = the rank at the position the query counts from, where
//            w0, w1 are the line's first two u32 words and up says q lies in the upper half.
// The arithmetic is modulo 2^64: offset may exceed the anchor rank when delta carries a negative
// bias (paired superblocks), and the sum is still exact.
struct BR16 {
    static constexpr int ID = QR_LAYOUT_16;
    static constexpr uint32_t HDR = 16, DATA = 1008, MID = 512;
    static constexpr bool QUARTER = false;
    static constexpr uint64_t SB_LINES = 64;     // lines per superblock
    static constexpr uint32_t SB_LOG = 6;
    static constexpr uint32_t SHIFT = 10;
    static constexpr uint64_t MAGIC = 0x8208208208208209ull;  // ceil(2^73 / 1008)
    static constexpr uint32_t MAGIC_T = 9;
    static constexpr uint64_t MAX_N = (1ull << 42) - 1;
    using Super = uint32_t;
    __device__ __forceinline__ static uint64_t offset(const Super *__restrict__ s, uint64_t j) {
        return (uint64_t)s[j >> SB_LOG] << SHIFT;
    }
    __device__ __forceinline__ static uint64_t delta(uint32_t w0, uint32_t, bool, uint64_t) { return w0 & 0xffffu; }
};

// Paired superblocks (the pairing variant of the paper's appendix on pairing superblocks): one
// shifted offset per 128 lines, taken at the pair's middle (line 64 of the 128) instead of its
// start, so the offset array is half as long.  Lines of the lower half store their delta plus
// BIAS = 64 * 1008 - 496 (the most bits between a lower line's middle and the pair's middle), which
// keeps it non-negative; the query removes BIAS again.
//   b_j = rank(1008 j + 496) - 2^10 s'_{j/128} + [j mod 128 < 64] BIAS
//   s'_i = floor(rank(1008 (128 i + 64)) / 2^10)
//   bounds: lower lines 0 <= b_j <= BIAS + 1023 = 65039; upper lines b_j <= 63*1008 + 496 + 1023
struct BR16P {
    static constexpr int ID = QR_LAYOUT_16P;
    static constexpr uint32_t HDR = 16, DATA = 1008, MID = 512;
    static constexpr bool QUARTER = false;
    static constexpr uint64_t SB_LINES = 128;
    static constexpr uint32_t SB_LOG = 7;
    static constexpr uint32_t SHIFT = 10;
    static constexpr uint64_t BIAS = 64 * 1008 - 496;
    static constexpr uint64_t MAGIC = BR16::MAGIC;
    static constexpr uint32_t MAGIC_T = BR16::MAGIC_T;
    static constexpr uint64_t MAX_N = (1ull << 42) - 1;
    using Super = uint32_t;
    __device__ __forceinline__ static uint64_t offset(const Super *__restrict__ s, uint64_t j) {
        return (uint64_t)s[j >> SB_LOG] << SHIFT;
    }
    __device__ __forceinline__ static uint64_t delta(uint32_t w0, uint32_t, bool, uint64_t j) {
        return (uint64_t)(w0 & 0xffffu) - ((j & 64u) ? 0ull : BIAS);
    }
};

// 32-bit inline deltas: floor(x/992) = mulhi(x, ceil(2^73/992)) >> 9, exact for x < 2^63
// (e = m*992 - 2^73 = 736 < 992, Granlund-Montgomery).
struct BR32 {
    static constexpr int ID = QR_LAYOUT_32;
    static constexpr uint32_t HDR = 32, DATA = 992, MID = 512;
    static constexpr bool QUARTER = false;
    static constexpr uint64_t SB_LINES = 1ull << 22;
    static constexpr uint32_t SB_LOG = 22;
    static constexpr uint32_t SHIFT = 0;
    static constexpr uint64_t MAGIC = 0x8421084210842109ull;  // ceil(2^73 / 992)
    static constexpr uint32_t MAGIC_T = 9;
    static constexpr uint64_t MAX_N = (1ull << 48) - 1;
    using Super = uint64_t;
    __device__ __forceinline__ static uint64_t offset(const Super *__restrict__ s, uint64_t j) { return s[j >> SB_LOG]; }
    __device__ __forceinline__ static uint64_t delta(uint32_t w0, uint32_t, bool, uint64_t) { return w0; }
};

// The paper's BiRank64: the line's first 64 bits hold the absolute rank at its middle, so there is
// no offset array at all.  960 data bits per line; the middle is data bit 448 (line bit 512).
// floor(x/960) = mulhi(x, ceil(2^73/960)) >> 9, exact for x < 2^63 (e = 448 < 960).
struct BR64 {
    static constexpr int ID = QR_LAYOUT_64;
    static constexpr uint32_t HDR = 64, DATA = 960, MID = 512;
    static constexpr bool QUARTER = false;
    static constexpr uint64_t SB_LINES = 0;  // no offset array
    static constexpr uint32_t SB_LOG = 0;
    static constexpr uint32_t SHIFT = 0;
    static constexpr uint64_t MAGIC = 0x8888888888888889ull;  // ceil(2^73 / 960)
    static constexpr uint32_t MAGIC_T = 9;
    static constexpr uint64_t MAX_N = (1ull << 48) - 1;
    using Super = uint64_t;
    __device__ __forceinline__ static uint64_t offset(const Super *__restrict__, uint64_t) { return 0; }
    __device__ __forceinline__ static uint64_t delta(uint32_t w0, uint32_t w1, bool, uint64_t) {
        return (uint64_t)w0 | ((uint64_t)w1 << 32);
    }
};

// The paper's BiRank16x2: two 16-bit deltas, to a quarter and to three quarters into the line (line
// bits 256 and 768), so a query popcounts at most a quarter line (256 bits) instead of a half.
// 992 data bits (bits [32, 1024)); superblocks of 64 lines with a shifted 32-bit offset as BR16.
//   line bits [0,16): rank(992 j + 224) - 2^10 s_{j/64};  [16,32): rank(992 j + 736) - 2^10 s_{j/64}
//   bounds: <= 63*992 + 736 + 1023 = 64255 < 2^16; s < 2^32 for n < 2^42
struct BR16X2 {
    static constexpr int ID = QR_LAYOUT_16X2;
    static constexpr uint32_t HDR = 32, DATA = 992, MID = 512;
    static constexpr bool QUARTER = true;
    static constexpr uint64_t SB_LINES = 64;
    static constexpr uint32_t SB_LOG = 6;
    static constexpr uint32_t SHIFT = 10;
    static constexpr uint64_t MAGIC = BR32::MAGIC;
    static constexpr uint32_t MAGIC_T = BR32::MAGIC_T;
    static constexpr uint64_t MAX_N = (1ull << 42) - 1;
    using Super = uint32_t;
    __device__ __forceinline__ static uint64_t offset(const Super *__restrict__ s, uint64_t j) {
        return (uint64_t)s[j >> SB_LOG] << SHIFT;
    }
    __device__ __forceinline__ static uint64_t delta(uint32_t w0, uint32_t, bool up, uint64_t) {
        return up ? (w0 >> 16) : (w0 & 0xffffu);
    }
};

template <class L>
__host__ __device__ __forceinline__ uint64_t line_of(uint64_t q) {
    return mulhi64(q, L::MAGIC) >> L::MAGIC_T;
}

// Masked popcount of one 512-bit half line given as 16 u32 words.  Counts positions [0, t) of the
// half when `upper`, and positions [t, 512) otherwise.
__device__ __forceinline__ uint32_t half_count(const uint32_t (&h)[16], uint32_t t, bool upper) {
    const uint32_t inv = upper ? 0u : 0xffffffffu;
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) c += __popc(h[k] & (prefix_mask32(t, k) ^ inv));
    return c;
}

// Popcount of the range a query counts inside the 512-bit half (16 u32 words) that holds q, with
// t = q's bit position in that half; fwd says whether the range follows the anchor (add it) or
// precedes it (subtract it).  Middle-anchored layouts count between t and the half's boundary with
// the middle; quarter-anchored layouts count between t and bit 256 of the half, one quarter line.
template <class L>
__device__ __forceinline__ uint32_t br_count(const uint32_t (&h)[16], uint32_t t, bool up, bool &fwd) {
    if constexpr (L::QUARTER) {
        fwd = t >= 256;
        const uint32_t u = t & 255u, inv = fwd ? 0u : 0xffffffffu;
        uint32_t c = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) c += __popc((fwd ? h[8 + k] : h[k]) & (prefix_mask32(u, k) ^ inv));
        return c;
    } else {
        fwd = up;
        return half_count(h, t, up);
    }
}

// rank(q) and the bit t_q of a BiRank layout, read by one lane: the half line that holds q and, for
// the upper half, the line's first two words (the header).  Requires q < n, so that t_q exists.
template <class L>
__device__ __forceinline__ uint64_t br_rank_bit(const uint4 *__restrict__ lines, const typename L::Super *__restrict__ super,
                                                uint64_t q, uint32_t &bit) {
    const uint64_t j = line_of<L>(q);
    const uint32_t p = (uint32_t)(q - j * L::DATA) + L::HDR;
    const bool up = p >= L::MID;
    const uint4 *H = lines + j * 8 + (up ? 4 : 0);
    const uint4 a = H[0], b = H[1], c = H[2], d = H[3];
    const uint32_t h[16] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, c.y, c.z, c.w, d.x, d.y, d.z, d.w};
    const uint2 hw = up ? reinterpret_cast<const uint2 *>(lines)[j * 16] : make_uint2(a.x, a.y);
    const uint32_t t = up ? p - L::MID : p;
    uint32_t w = 0;  // the word holding bit t, picked with masks (no indexed register array)
#pragma unroll
    for (uint32_t k = 0; k < 16; ++k) w |= h[k] & ((t >> 5) == k ? 0xffffffffu : 0u);
    bit = (w >> (t & 31u)) & 1u;
    bool fwd;
    const uint32_t cnt = br_count<L>(h, t, up, fwd);
    const uint64_t anchor = L::offset(super, j) + L::delta(hw.x, hw.y, up, j);
    return fwd ? anchor + cnt : anchor - cnt;
}

}  // namespace qr
