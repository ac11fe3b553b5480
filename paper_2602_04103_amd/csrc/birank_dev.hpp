// Device-side BiRank layout traits and a one-lane rank, shared by the BiRank kernels and by the
// FM-index's locate walk (which ranks over the bitvector of sampled suffix-array rows).  The layouts
// are described with the BiRank kernels.
#pragma once

#include "common.hpp"

namespace qr {

struct BR16 {
    static constexpr uint32_t HDR = 16, DATA = 1008, MID = 512;
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
    __device__ __forceinline__ static uint32_t delta(uint32_t w0) { return w0 & 0xffffu; }
};

// 32-bit inline deltas: floor(x/992) = mulhi(x, ceil(2^73/992)) >> 9, exact for x < 2^63
// (e = m*992 - 2^73 = 736 < 992, Granlund-Montgomery).
struct BR32 {
    static constexpr uint32_t HDR = 32, DATA = 992, MID = 512;
    static constexpr uint64_t SB_LINES = 1ull << 22;
    static constexpr uint32_t SB_LOG = 22;
    static constexpr uint32_t SHIFT = 0;
    static constexpr uint64_t MAGIC = 0x8421084210842109ull;  // ceil(2^73 / 992)
    static constexpr uint32_t MAGIC_T = 9;
    static constexpr uint64_t MAX_N = (1ull << 48) - 1;
    using Super = uint64_t;
    __device__ __forceinline__ static uint64_t offset(const Super *__restrict__ s, uint64_t j) { return s[j >> SB_LOG]; }
    __device__ __forceinline__ static uint32_t delta(uint32_t w0) { return w0; }
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

// rank(q) and the bit t_q of a BiRank layout, read by one lane: the half line that holds q and, for
// the upper half, the line's first word (the delta).  Requires q < n, so that t_q exists.
template <class L>
__device__ __forceinline__ uint64_t br_rank_bit(const uint4 *__restrict__ lines, const typename L::Super *__restrict__ super,
                                                uint64_t q, uint32_t &bit) {
    const uint64_t j = line_of<L>(q);
    const uint32_t p = (uint32_t)(q - j * L::DATA) + L::HDR;
    const bool up = p >= L::MID;
    const uint4 *H = lines + j * 8 + (up ? 4 : 0);
    const uint4 a = H[0], b = H[1], c = H[2], d = H[3];
    const uint32_t h[16] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, c.y, c.z, c.w, d.x, d.y, d.z, d.w};
    const uint32_t hdr = up ? reinterpret_cast<const uint32_t *>(lines)[j * 32] : a.x;
    const uint32_t t = up ? p - L::MID : p;
    uint32_t w = 0;  // the word holding bit t, picked with masks (no indexed register array)
#pragma unroll
    for (uint32_t k = 0; k < 16; ++k) w |= h[k] & ((t >> 5) == k ? 0xffffffffu : 0u);
    bit = (w >> (t & 31u)) & 1u;
    const uint32_t cnt = half_count(h, t, up);
    const uint64_t mid = L::offset(super, j) + L::delta(hdr);
    return up ? mid + cnt : mid - cnt;
}

}  // namespace qr
