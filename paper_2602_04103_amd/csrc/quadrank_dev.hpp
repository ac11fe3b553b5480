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

__device__ __forceinline__ uint32_t sel4(const uint4 &v, uint32_t c) {
    return c == 0 ? v.x : c == 1 ? v.y : c == 2 ? v.z : v.w;
}

__device__ __forceinline__ uint32_t delta_of(const HalfLine &hl, uint32_t c) {
    const uint32_t d = (c & 2) ? hl.dGT : hl.dAC;
    return (c & 1) ? (d >> 16) : (d & 0xffffu);
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

}  // namespace qr
