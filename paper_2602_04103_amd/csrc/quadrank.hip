// QuadRank on gfx950 (paper Section 4): DNA rank with four deltas inlined per 128-byte line and
// the text stored transposed (a plane of low bits and a plane of high bits).
//
// Line j = 16 little-endian u64 words = 8 pairs (lo_k, hi_k) = (word 2k, word 2k+1), k = 0..7.
// Pair k holds line base slots [64k, 64k+64): bit b of lo_k / hi_k is the low / high bit of slot
// 64k + b.  The first HDR slots hold the deltas instead of bases; the rest hold DATA bases
// (slot = base - DATA j + HDR).  The line's middle is slot 256, so each half line (pairs 0-3 or
// 4-7) is one 64-byte segment, and a query counts at most 256 slots.
//
//   QR16 (default; the paper's QuadRank16 re-derived for 128-byte lines): HDR = 32 slots,
//     lo_0 bits [0,16) = b_A, [16,32) = b_C; hi_0 bits [0,16) = b_G, [16,32) = b_T (the listing's
//     delta placement c + (c&2) in u16 units); DATA = 480; middle = base 224;
//     b_{j,c} = rank(480 j + 224, c) - 2^12 s_{j/128, c};  s_{i,c} = floor(rank(61440 i, c) / 2^12)
//     bounds: b <= 127*480 + 224 + 4095 = 65279 < 2^16; s < 2^32 for n < 2^44
//   QR32 (a 32-bit inline variant): HDR = 64 slots, lo_0 = b_A | b_C << 32, hi_0 = b_G | b_T << 32;
//     DATA = 448; middle = base 192; b_{j,c} = rank(448 j + 192, c) - s_{j/2^23, c} (s exact, u64)
//     bounds: b <= (2^23 - 1)*448 + 192 < 2^32
//   QR16P (QR16 with paired superblocks), QR64 (the paper's QuadRank64: absolute u64 ranks, no
//   offset array) and QR24_8 (the paper's QuadRank24_8 on 128-byte lines: three anchors per line, a
//   query counts at most 64 bases) are defined, with their bounds, beside their layout traits
//   (quadrank_dev.hpp)
//
// floor(n/DATA) + 1 lines; bases past n are stored as A (code 0) and every delta is taken over that
// padded text, so the padding cancels for every q <= n.
//
// Query: j = floor(q/DATA), p = q - DATA j + HDR (slot of q);
//   rank(q,c) = offset_{j,c} + b_{j,c} + #c in slots [256, p)   if p >= 256
//   rank(q,c) = offset_{j,c} + b_{j,c} - #c in slots [p, 256)   if p <  256
// Symbol c matches where (lo XNOR c_0) AND (hi XNOR c_1).  rank4 counts the range once per
// plane: T = |lo&hi|, C = |lo| - T, G = |hi| - T, A = len - T - C - G.
#include <algorithm>
#include <new>

#include "common.hpp"
#include "quadrank_dev.hpp"
#include "sweep.hpp"

using namespace qr;

struct qr_quadrank_s {
    int device;
    int layout;  // QR_LAYOUT_16, _32, _16P, _64 or _24_8
    uint64_t n, n_lines, n_sb;
    uint64_t *lines;  // n_lines * 16 words
    void *super;      // n_sb * 4 offsets: u32 (16-bit layouts) or u64 (32-bit and 24_8 layouts); none for QR64
    uint32_t *err;
    qr_tuning tune;
};

namespace {

constexpr uint32_t GROUP_LINES = 128;  // lines per build workgroup (QR16: one superblock)

__device__ __forceinline__ uint64_t masked_packed(const uint64_t *__restrict__ packed, uint64_t w, uint64_t n,
                                                  uint64_t n_words) {
    if (w >= n_words) return 0;
    uint64_t x = packed[w];
    uint64_t first = w * 32;
    if (first + 32 > n) x &= (1ull << (2 * (n - first))) - 1ull;  // n - first in [1, 31]
    return x;
}

// C, G, T counts of a packed word (A is implied by the length).
__device__ __forceinline__ void word_counts(uint64_t x, uint32_t &cC, uint32_t &cG, uint32_t &cT) {
    const uint64_t lo = x & 0x5555555555555555ull, hi = (x >> 1) & 0x5555555555555555ull;
    const uint32_t t = __popcll(lo & hi);
    cT += t;
    cC += __popcll(lo) - t;
    cG += __popcll(hi) - t;
}

// Pass 1: symbol counts of each group of 128 lines (padded with A), one wavefront per group and
// COUNT_GROUPS groups per workgroup.  Groups made only of whole packed words below n are read with
// 16-byte loads when the input is 16-byte aligned; the last group, or an input aligned to 8 bytes
// only, takes the masked word path.
constexpr uint32_t COUNT_GROUPS = 4;

template <class L>
__global__ __launch_bounds__(64 * COUNT_GROUPS) void qr_count_kernel(const uint64_t *__restrict__ packed, uint64_t n,
                                                                     uint64_t n_words, uint64_t n_groups,
                                                                     uint32_t *__restrict__ cnt) {
    constexpr uint32_t W = GROUP_LINES * L::WORDS;
    static_assert(W % 2 == 0, "a group must be a whole number of 16-byte chunks");
    const uint64_t g = (uint64_t)blockIdx.x * COUNT_GROUPS + threadIdx.x / 64;
    if (g >= n_groups) return;
    const uint32_t lane = __lane_id();
    const uint64_t w0 = g * W;
    uint32_t cC = 0, cG = 0, cT = 0;
    if (((uintptr_t)packed & 15) == 0 && w0 + W <= n / 32) {
        const uint4 *v = reinterpret_cast<const uint4 *>(packed + w0);
#pragma unroll 4
        for (uint32_t k = lane; k < W / 2; k += 64) {
            const uint4 x = v[k];
            word_counts((uint64_t)x.x | ((uint64_t)x.y << 32), cC, cG, cT);
            word_counts((uint64_t)x.z | ((uint64_t)x.w << 32), cC, cG, cT);
        }
    } else {
        for (uint32_t k = lane; k < W; k += 64) word_counts(masked_packed(packed, w0 + k, n, n_words), cC, cG, cT);
    }
    cC = wave_sum(cC), cG = wave_sum(cG), cT = wave_sum(cT);
    if (lane == 0) {
        cnt[4 * g + 0] = GROUP_LINES * L::DATA - cC - cG - cT;
        cnt[4 * g + 1] = cC;
        cnt[4 * g + 2] = cG;
        cnt[4 * g + 3] = cT;
    }
}

// Exact offsets (QR32, QR24_8): s_{i,c} = the rank at the first line of superblock i, which is the
// first line of build group gps * i (gps = groups per superblock).
__global__ void qr_exact_super_kernel(const uint64_t *__restrict__ base, uint64_t n_groups, uint64_t n_sb, uint64_t gps,
                                      uint64_t *__restrict__ super) {
    const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < 4 * n_sb) super[e] = base[4 * std::min((e / 4) * gps, n_groups - 1) + (e & 3)];
}

// Offsets of paired superblocks (QR16P): s'_{i,c} = the rank at the start of group 2i + 1 (the
// pair's middle), shifted; a last pair without its upper group takes the rank after its lower
// group, whose counts cover all of its (A-padded) lines.
__global__ void qr_paired_super_kernel(const uint64_t *__restrict__ base, const uint32_t *__restrict__ cnt,
                                       uint64_t n_groups, uint64_t n_sb, uint32_t shift, uint32_t *__restrict__ super) {
    const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 4 * n_sb) return;
    const uint64_t g = 2 * (e / 4) + 1, c = e & 3;
    const uint64_t r = g < n_groups ? base[4 * g + c] : base[4 * (g - 1) + c] + cnt[4 * (g - 1) + c];
    super[e] = (uint32_t)(r >> shift);
}

// Pass 3: one 128-lane workgroup per group; lane t forms line 128 g + t from packed words
// [WORDS t, WORDS t + WORDS) of the group.
constexpr int OUT_STRIDE = 17;

template <class L>
__global__ __launch_bounds__(128) void qr_write_kernel(const uint64_t *__restrict__ packed, uint64_t n,
                                                       uint64_t n_words, const uint64_t *__restrict__ base,
                                                       const uint32_t *__restrict__ paired_super, uint64_t n_lines,
                                                       uint64_t *__restrict__ lines) {
    constexpr uint32_t W = GROUP_LINES * L::WORDS;
    // packed words before the anchor(s): the lower half for middle-anchored layouts; for QR24_8 the
    // words before data bases 64, 192 and 320 (slots 192, 320, 448)
    constexpr uint32_t FIRST = L::MULTI ? 2 : (L::MID - L::HDR) / 32;
    constexpr uint32_t SECOND = L::MULTI ? 6 : FIRST, THIRD = L::MULTI ? 10 : FIRST;
    constexpr uint64_t GPS = L::SB_LINES >= GROUP_LINES ? L::SB_LINES / GROUP_LINES : 1;  // groups per superblock
    // one LDS buffer holds the group's input words, then (after a barrier) the staged output lines
    constexpr uint32_t BUF = (W > 128 * OUT_STRIDE) ? W : 128 * OUT_STRIDE;
    __shared__ __align__(16) uint64_t buf[BUF];
    __shared__ uint64_t wave_tot[2];
    uint64_t *in = buf, *stage = buf;
    const uint64_t g = blockIdx.x;
    const int t = threadIdx.x;
    if (((uintptr_t)packed & 15) == 0 && g * W + W <= n / 32) {  // whole words only: 16-byte loads
        const uint4 *v = reinterpret_cast<const uint4 *>(packed + g * W);
        uint4 *d = reinterpret_cast<uint4 *>(in);
#pragma unroll 4
        for (uint32_t k = t; k < W / 2; k += 128) d[k] = v[k];
    } else {
        for (uint32_t k = t; k < W; k += 128) in[k] = masked_packed(packed, g * W + k, n, n_words);
    }
    __syncthreads();

    uint32_t lo[L::WORDS], hi[L::WORDS];
    uint32_t fC = 0, fG = 0, fT = 0, aC = 0, aG = 0, aT = 0;  // counts before the (first) anchor, whole line
    uint32_t sC = 0, sG = 0, sT = 0, tC = 0, tG = 0, tT = 0;  // QR24_8: words [FIRST, SECOND), [SECOND, THIRD)
#pragma unroll
    for (int k = 0; k < (int)L::WORDS; ++k) {
        const uint64_t x = in[L::WORDS * t + k];
        lo[k] = even_bits(x);
        hi[k] = even_bits(x >> 1);
        if (k < (int)FIRST) word_counts(x, fC, fG, fT);
        if (L::MULTI && k >= (int)FIRST && k < (int)SECOND) word_counts(x, sC, sG, sT);
        if (L::MULTI && k >= (int)SECOND && k < (int)THIRD) word_counts(x, tC, tG, tT);
        word_counts(x, aC, aG, aT);
    }
    const uint32_t fA = 32 * FIRST - fC - fG - fT, aA = L::DATA - aC - aG - aT;
    // Exclusive scan of the four line totals over the 128 lines; each stays below 2^16 over a
    // group (<= 128 * 480), so the four are packed into one u64 and scanned together.
    const uint64_t tot = (uint64_t)aA | ((uint64_t)aC << 16) | ((uint64_t)aG << 32) | ((uint64_t)aT << 48);
    uint64_t incl = wave_inclusive_scan<uint64_t>(tot);
    if (__lane_id() == 63) wave_tot[t / 64] = incl;
    __syncthreads();
    if (t >= 64) incl += wave_tot[0];
    const uint64_t before = incl - tot;
    const uint32_t first[4] = {fA, fC, fG, fT};
    uint64_t d[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        uint64_t off = 0;  // the offset the query reconstructs
        if constexpr (L::ID == QR_LAYOUT_16P) {
            off = ((uint64_t)paired_super[4 * (g >> 1) + c] << L::SHIFT) - ((g & 1) ? 0ull : L::BIAS);
        } else if constexpr (L::SB_LINES != 0) {
            const uint64_t sb_base = base[4 * ((g / GPS) * GPS) + c];
            off = (sb_base >> L::SHIFT) << L::SHIFT;
        }
        d[c] = base[4 * g + c] - off + ((before >> (16 * c)) & 0xffffu) + first[c];
    }

    uint64_t o[16];
    if constexpr (L::MULTI) {  // u32 word c: L1_c | d1_c << 24; u32 word 4 + c: d2_c
        const uint32_t d1[4] = {32 * (SECOND - FIRST) - sC - sG - sT, sC, sG, sT};
        const uint32_t d2[4] = {32 * (THIRD - SECOND) - tC - tG - tT, tC, tG, tT};
        uint32_t w[8];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            w[c] = (uint32_t)d[c] | (d1[c] << 24);
            w[4 + c] = d2[c];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) o[k] = (uint64_t)w[2 * k] | ((uint64_t)w[2 * k + 1] << 32);
    }
    if constexpr (L::HDR == 128) {  // header in pairs 0 and 1; pair k >= 2 holds packed words 2k-4, 2k-3
        if constexpr (!L::MULTI) {  // QR64: the absolute ranks of A, C, G, T as u64 words 0..3
#pragma unroll
            for (int c = 0; c < 4; ++c) o[c] = d[c];
        }
#pragma unroll
        for (int k = 2; k < 8; ++k) {
            o[2 * k] = (uint64_t)lo[2 * k - 4] | ((uint64_t)lo[2 * k - 3] << 32);
            o[2 * k + 1] = (uint64_t)hi[2 * k - 4] | ((uint64_t)hi[2 * k - 3] << 32);
        }
    } else if constexpr (L::HDR == 32) {  // deltas in the low 32 slots of pair 0, bases 0..31 in its high 32 slots
        o[0] = (d[0] | (d[1] << 16)) | ((uint64_t)lo[0] << 32);
        o[1] = (d[2] | (d[3] << 16)) | ((uint64_t)hi[0] << 32);
#pragma unroll
        for (int k = 1; k < 8; ++k) {
            o[2 * k] = (uint64_t)lo[2 * k - 1] | ((uint64_t)lo[2 * k] << 32);
            o[2 * k + 1] = (uint64_t)hi[2 * k - 1] | ((uint64_t)hi[2 * k] << 32);
        }
    } else {  // QR32: deltas fill pair 0; pair k >= 1 holds packed words 2k-2 and 2k-1
        o[0] = d[0] | (d[1] << 32);
        o[1] = d[2] | (d[3] << 32);
#pragma unroll
        for (int k = 1; k < 8; ++k) {
            o[2 * k] = (uint64_t)lo[2 * k - 2] | ((uint64_t)lo[2 * k - 1] << 32);
            o[2 * k + 1] = (uint64_t)hi[2 * k - 2] | ((uint64_t)hi[2 * k - 1] << 32);
        }
    }
    __syncthreads();  // every lane has read its input words: the buffer now takes the output
#pragma unroll
    for (int k = 0; k < 16; ++k) stage[t * OUT_STRIDE + k] = o[k];
    __syncthreads();
    const uint64_t l0 = g * GROUP_LINES;
    const uint32_t nl = (uint32_t)std::min<uint64_t>(GROUP_LINES, n_lines - l0);
    uint4 *dst = reinterpret_cast<uint4 *>(lines + l0 * 16);
    for (uint32_t e = t; e < nl * 8; e += 128) {
        const uint64_t *src = stage + (e >> 3) * OUT_STRIDE + (e & 7) * 2;
        uint64_t a = src[0], b = src[1];
        dst[e] = make_uint4((uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32));
    }
}

// ---- one lane per query (lanes = 1) --------------------------------------------------------------
template <class L>
__device__ __forceinline__ void load_lane_half(const uint4 *__restrict__ lines, uint64_t q, PairHalf &ph, uint4 &hdr,
                                               uint4 &hdr1) {
    ph.j = qline_of<L>(q);
    const uint32_t p = (uint32_t)(q - ph.j * L::DATA) + L::HDR;
    ph.up = p >= L::MID;
    ph.t = ph.up ? p - L::MID : p;
    const uint4 *H = lines + ph.j * 8 + (ph.up ? 4 : 0);
    const uint4 a = H[0], b = H[1], c = H[2], d = H[3];
    ph.w[0] = a.x, ph.w[1] = a.y, ph.w[2] = a.z, ph.w[3] = a.w;
    ph.w[4] = b.x, ph.w[5] = b.y, ph.w[6] = b.z, ph.w[7] = b.w;
    ph.w[8] = c.x, ph.w[9] = c.y, ph.w[10] = c.z, ph.w[11] = c.w;
    ph.w[12] = d.x, ph.w[13] = d.y, ph.w[14] = d.z, ph.w[15] = d.w;
    // The header: u32 words 0..3 of the line, and words 4..7 for the layouts with 128 header slots.
    // Those layouts read it from the line in both halves: selecting between that load and the
    // register copies a, b would be compiled into a load through stack copies of a and b.
    if constexpr (L::HDR > 64) {
        hdr = lines[ph.j * 8];
        hdr1 = lines[ph.j * 8 + 1];
    } else {
        hdr = ph.up ? lines[ph.j * 8] : a;
        hdr1 = make_uint4(0u, 0u, 0u, 0u);
    }
}

// The line slot of q from its half and the slot inside it.
__device__ __forceinline__ uint32_t line_slot(const PairHalf &ph) { return ph.up ? ph.t + QR_MID : ph.t; }

// rank(q, c) (PREFIX = false) or prefix_rank(q, c) = #{i < q : t_i <= c} (PREFIX = true): the same
// walk with the symbol test, the delta and the offset replaced by their sums over the symbols <= c.
template <class L, int PER_LANE, bool PREFIX>
__device__ __forceinline__ void sym_lane_body(const uint4 *__restrict__ lines, const typename L::Super *__restrict__ super,
                                              uint64_t n, const uint64_t *__restrict__ Q,
                                              const uint8_t *__restrict__ Cs, uint64_t nq, uint64_t *__restrict__ out,
                                              uint32_t *__restrict__ err) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i0 < nq; i0 += stride * PER_LANE) {
        uint64_t q[PER_LANE], off[PER_LANE], r[PER_LANE];
        uint32_t c[PER_LANE];
        bool bad[PER_LANE];
        PairHalf ph[PER_LANE];
        uint4 hdr[PER_LANE], hdr1[PER_LANE];
#pragma unroll
        for (int u = 0; u < PER_LANE; ++u) {
            const uint64_t i = min(i0 + u * stride, nq - 1);
            q[u] = load_once(Q + i);
            c[u] = load_once(Cs + i);
        }
#pragma unroll
        for (int u = 0; u < PER_LANE; ++u) {
            bad[u] = q[u] > n || c[u] > 3;
            load_lane_half<L>(lines, bad[u] ? 0 : q[u], ph[u], hdr[u], hdr1[u]);
            off[u] = PREFIX ? offset_le<L>(super, ph[u].j, c[u] & 3u) : L::offset1(super, ph[u].j, c[u] & 3u);
        }
#pragma unroll
        for (int u = 0; u < PER_LANE; ++u) {
            const uint32_t cc = c[u] & 3u, hu = (uint32_t)ph[u].up;
            bool fwd;
            const uint32_t cnt = PREFIX ? count_le<L>(ph[u], hu, cc, fwd) : count1<L>(ph[u], hu, cc, fwd);
            const uint32_t p = line_slot(ph[u]);
            const uint64_t d = PREFIX ? delta_le<L>(hdr[u], hdr1[u], cc, p, ph[u].j)
                                      : L::delta(hdr[u], hdr1[u], cc, p, ph[u].j);
            const uint64_t anchor = off[u] + d;
            r[u] = bad[u] ? ~0ull : (fwd ? anchor + cnt : anchor - cnt);
        }
#pragma unroll
        for (int u = 0; u < PER_LANE; ++u) {
            const uint64_t i = i0 + u * stride;
            if (i < nq) {
                store_once(out + i, r[u]);
                if (bad[u]) atomicOr(err, 1u);
            }
        }
    }
}

#define QR_SYM_ARGS                                                                                              \
    const uint4 *__restrict__ lines, const typename L::Super *__restrict__ super, uint64_t n,                    \
        const uint64_t *__restrict__ Q, const uint8_t *__restrict__ Cs, uint64_t nq, uint64_t *__restrict__ out, \
        uint32_t *__restrict__ err

template <class L, int PER_LANE>
__global__ __launch_bounds__(256) void qr_rank1_kernel(QR_SYM_ARGS) {
    sym_lane_body<L, PER_LANE, false>(lines, super, n, Q, Cs, nq, out, err);
}

template <class L, int PER_LANE>
__global__ __launch_bounds__(256) void qr_prefix_kernel(QR_SYM_ARGS) {
    sym_lane_body<L, PER_LANE, true>(lines, super, n, Q, Cs, nq, out, err);
}

template <class L, int PER_LANE>
__global__ __launch_bounds__(256) void qr_rank4_kernel(const uint4 *__restrict__ lines,
                                                       const typename L::Super *__restrict__ super, uint64_t n,
                                                       const uint64_t *__restrict__ Q, uint64_t nq,
                                                       uint64_t *__restrict__ out4, uint32_t *__restrict__ err) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i0 < nq; i0 += stride * PER_LANE) {
        uint64_t q[PER_LANE];
        bool bad[PER_LANE];
        PairHalf ph[PER_LANE];
        uint4 hdr[PER_LANE], hdr1[PER_LANE];
        uint64_t off[PER_LANE][4];
#pragma unroll
        for (int u = 0; u < PER_LANE; ++u) q[u] = load_once(Q + min(i0 + u * stride, nq - 1));
#pragma unroll
        for (int u = 0; u < PER_LANE; ++u) {
            bad[u] = q[u] > n;
            load_lane_half<L>(lines, bad[u] ? 0 : q[u], ph[u], hdr[u], hdr1[u]);
            L::offset4(super, ph[u].j, off[u]);
        }
#pragma unroll
        for (int u = 0; u < PER_LANE; ++u) {
            uint32_t cnt[4];
            bool fwd;
            count4<L>(ph[u], (uint32_t)ph[u].up, cnt, fwd);
            const uint32_t p = line_slot(ph[u]);
            uint64_t r[4];
#pragma unroll
            for (uint32_t cc = 0; cc < 4; ++cc) {
                const uint64_t anchor = off[u][cc] + L::delta(hdr[u], hdr1[u], cc, p, ph[u].j);
                r[cc] = bad[u] ? ~0ull : (fwd ? anchor + cnt[cc] : anchor - cnt[cc]);
            }
            const uint64_t i = i0 + u * stride;
            if (i < nq) {
                store_once2(out4 + 4 * i, r[0], r[1]);
                store_once2(out4 + 4 * i + 2, r[2], r[3]);
                if (bad[u]) atomicOr(err, 1u);
            }
        }
    }
}

// ---- lane pairs (default) --------------------------------------------------------------------------
// Lanes 2k, 2k+1 serve one query, lane hf loading half hf of the line (64 contiguous bytes), so each
// wave load instruction touches 32 lines.  The lane holding q's half counts; lane 0 adds offset and
// delta; the two contributions are summed across the pair.
// rank(q[u], c[u]) (or the count of symbols <= c[u] when PREFIX) for one query per unroll slot u,
// valid in both lanes of the pair; bad[u] marks q > n or c > 3 (result UINT64_MAX).
template <class L, int PER_PAIR, bool PREFIX>
__device__ __forceinline__ void sym_pair_compute(const uint4 *__restrict__ lines,
                                                 const typename L::Super *__restrict__ super, uint64_t n,
                                                 const uint64_t (&q)[PER_PAIR], const uint32_t (&c)[PER_PAIR],
                                                 uint32_t hf, uint64_t (&r)[PER_PAIR], bool (&bad)[PER_PAIR]) {
    uint64_t off[PER_PAIR];
    PairHalf ph[PER_PAIR];
#pragma unroll
    for (int u = 0; u < PER_PAIR; ++u) {
        bad[u] = q[u] > n || c[u] > 3;
        load_pair_half<L>(lines, bad[u] ? 0 : q[u], hf, ph[u]);
        off[u] = PREFIX ? offset_le<L>(super, ph[u].j, c[u] & 3u) : L::offset1(super, ph[u].j, c[u] & 3u);
    }
#pragma unroll
    for (int u = 0; u < PER_PAIR; ++u) {
        const uint32_t cc = c[u] & 3u;
        bool fwd;
        const uint32_t cnt = PREFIX ? count_le<L>(ph[u], hf, cc, fwd) : count1<L>(ph[u], hf, cc, fwd);
        uint64_t mine = fwd ? (uint64_t)cnt : 0ull - (uint64_t)cnt;
        if (hf == 0) {  // lane 0 holds the header (the first eight words of the line)
            const uint32_t p = line_slot(ph[u]);
            const uint4 a = hdr_lo(ph[u].w), b = hdr_hi(ph[u].w);
            mine += off[u] + (PREFIX ? delta_le<L>(a, b, cc, p, ph[u].j) : L::delta(a, b, cc, p, ph[u].j));
        }
        r[u] = bad[u] ? ~0ull : mine + pair_swap64(mine);
    }
}

template <class L, int PER_PAIR, bool PREFIX>
__device__ __forceinline__ void sym_pair_body(const uint4 *__restrict__ lines, const typename L::Super *__restrict__ super,
                                              uint64_t n, const uint64_t *__restrict__ Q,
                                              const uint8_t *__restrict__ Cs, uint64_t nq, uint64_t *__restrict__ out,
                                              uint32_t *__restrict__ err) {
    const uint32_t hf = threadIdx.x & 1u;
    const uint64_t pairs = ((uint64_t)gridDim.x * blockDim.x) >> 1;
    for (uint64_t i0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 1; i0 < nq; i0 += pairs * PER_PAIR) {
        uint64_t q[PER_PAIR], r[PER_PAIR];
        uint32_t c[PER_PAIR];
        bool bad[PER_PAIR];
#pragma unroll
        for (int u = 0; u < PER_PAIR; ++u) {
            const uint64_t i = min(i0 + u * pairs, nq - 1);
            q[u] = load_once(Q + i);
            c[u] = load_once(Cs + i);
        }
        sym_pair_compute<L, PER_PAIR, PREFIX>(lines, super, n, q, c, hf, r, bad);
#pragma unroll
        for (int u = 0; u < PER_PAIR; ++u) {
            const uint64_t i = i0 + u * pairs;
            if (hf == 0 && i < nq) {
                store_once(out + i, r[u]);
                if (bad[u]) atomicOr(err, 1u);
            }
        }
    }
}

// Sweep form: one tile of 256*QPT queries per workgroup, answered in position order (sweep.hpp);
// results replace the sorted positions in LDS and are written back in query order.
template <class L, int PER_PAIR, bool PREFIX, int QPT>
__global__ __launch_bounds__(SWEEP_BLOCK) void qr_sym_sweep_kernel(QR_SYM_ARGS, uint32_t shift) {
    __shared__ SweepLds<QPT, true> S;
    constexpr uint32_t PAIRS = SWEEP_BLOCK / 2;
    const uint64_t base = (uint64_t)blockIdx.x * (SWEEP_BLOCK * QPT);
    const uint32_t m = (uint32_t)min<uint64_t>(SWEEP_BLOCK * QPT, nq - base);
    sweep_sort<QPT, true>(Q, Cs, base, m, shift, S);
    const uint32_t hf = threadIdx.x & 1u;
    for (uint32_t s0 = threadIdx.x >> 1; s0 < m; s0 += PAIRS * PER_PAIR) {
        uint64_t q[PER_PAIR], r[PER_PAIR];
        uint32_t c[PER_PAIR];
        bool bad[PER_PAIR];
#pragma unroll
        for (int u = 0; u < PER_PAIR; ++u) {
            const uint32_t sl = min(s0 + u * PAIRS, m - 1);  // slots past m: discarded, any value is safe
            q[u] = S.q[sl];
            c[u] = S.c[sl];
        }
        sym_pair_compute<L, PER_PAIR, PREFIX>(lines, super, n, q, c, hf, r, bad);
#pragma unroll
        for (int u = 0; u < PER_PAIR; ++u) {
            const uint32_t sl = s0 + u * PAIRS;
            if (hf == 0 && sl < m) {
                S.q[sl] = r[u];
                if (bad[u]) atomicOr(err, 1u);
            }
        }
    }
    __syncthreads();
    sweep_store<QPT, true>(out, base, m, S);
}

template <class L, int PER_PAIR>
__global__ __launch_bounds__(256) void qr_rank1_pair_kernel(QR_SYM_ARGS) {
    sym_pair_body<L, PER_PAIR, false>(lines, super, n, Q, Cs, nq, out, err);
}

template <class L, int PER_PAIR>
__global__ __launch_bounds__(256) void qr_prefix_pair_kernel(QR_SYM_ARGS) {
    sym_pair_body<L, PER_PAIR, true>(lines, super, n, Q, Cs, nq, out, err);
}

// rank4 of one query per unroll slot u: lane 0 ends with (A, C) in (ra, rb), lane 1 with (G, T).
template <class L, int PER_PAIR>
__device__ __forceinline__ void rank4_pair_compute(const uint4 *__restrict__ lines,
                                                   const typename L::Super *__restrict__ super, uint64_t n,
                                                   const uint64_t (&q)[PER_PAIR], uint32_t hf, uint64_t (&ra)[PER_PAIR],
                                                   uint64_t (&rb)[PER_PAIR], bool (&bad)[PER_PAIR]) {
    uint64_t off[PER_PAIR][4];
    PairHalf ph[PER_PAIR];
#pragma unroll
    for (int u = 0; u < PER_PAIR; ++u) {
        bad[u] = q[u] > n;
        load_pair_half<L>(lines, bad[u] ? 0 : q[u], hf, ph[u]);
        L::offset4(super, ph[u].j, off[u]);
    }
#pragma unroll
    for (int u = 0; u < PER_PAIR; ++u) {
        uint32_t cnt[4];
        bool fwd;
        count4<L>(ph[u], hf, cnt, fwd);
        const uint32_t p = line_slot(ph[u]);
        uint64_t r[4];
#pragma unroll
        for (uint32_t cc = 0; cc < 4; ++cc) {
            uint64_t mine = fwd ? (uint64_t)cnt[cc] : 0ull - (uint64_t)cnt[cc];
            if (hf == 0) mine += off[u][cc] + L::delta(hdr_lo(ph[u].w), hdr_hi(ph[u].w), cc, p, ph[u].j);
            r[cc] = mine + pair_swap64(mine);
        }
        // lane 0 writes symbols A, C and lane 1 writes G, T of the row
        ra[u] = bad[u] ? ~0ull : (hf == 0 ? r[0] : r[2]);
        rb[u] = bad[u] ? ~0ull : (hf == 0 ? r[1] : r[3]);
    }
}

template <class L, int PER_PAIR>
__global__ __launch_bounds__(256) void qr_rank4_pair_kernel(const uint4 *__restrict__ lines,
                                                            const typename L::Super *__restrict__ super, uint64_t n,
                                                            const uint64_t *__restrict__ Q, uint64_t nq,
                                                            uint64_t *__restrict__ out4, uint32_t *__restrict__ err) {
    const uint32_t hf = threadIdx.x & 1u;
    const uint64_t pairs = ((uint64_t)gridDim.x * blockDim.x) >> 1;
    for (uint64_t i0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 1; i0 < nq; i0 += pairs * PER_PAIR) {
        uint64_t q[PER_PAIR], ra[PER_PAIR], rb[PER_PAIR];
        bool bad[PER_PAIR];
#pragma unroll
        for (int u = 0; u < PER_PAIR; ++u) q[u] = load_once(Q + min(i0 + u * pairs, nq - 1));
        rank4_pair_compute<L, PER_PAIR>(lines, super, n, q, hf, ra, rb, bad);
#pragma unroll
        for (int u = 0; u < PER_PAIR; ++u) {
            const uint64_t i = i0 + u * pairs;
            if (i < nq) {
                store_once2(out4 + 4 * i + 2 * hf, ra[u], rb[u]);
                if (bad[u] && hf == 0) atomicOr(err, 1u);
            }
        }
    }
}

// Sweep form of rank4.  With tiles of 1024 queries the 32-byte rows are staged in LDS in query
// order (32 KB beside the 13 KB of the sort) and written back coalesced; with larger tiles, whose
// rows would not fit, each row goes straight to its own slot (a scatter: slower).
template <class L, int PER_PAIR, int QPT>
__global__ __launch_bounds__(SWEEP_BLOCK) void qr_rank4_sweep_kernel(const uint4 *__restrict__ lines,
                                                                     const typename L::Super *__restrict__ super,
                                                                     uint64_t n, const uint64_t *__restrict__ Q,
                                                                     uint64_t nq, uint64_t *__restrict__ out4,
                                                                     uint32_t *__restrict__ err, uint32_t shift) {
    constexpr bool STAGE = QPT <= 4;
    __shared__ SweepLds<QPT, false> S;
    __shared__ u64x2_t R[STAGE ? 2 * SWEEP_BLOCK * QPT : 1];  // half-row k of the tile's query k / 2
    constexpr uint32_t PAIRS = SWEEP_BLOCK / 2;
    const uint64_t base = (uint64_t)blockIdx.x * (SWEEP_BLOCK * QPT);
    const uint32_t m = (uint32_t)min<uint64_t>(SWEEP_BLOCK * QPT, nq - base);
    sweep_sort<QPT, false>(Q, nullptr, base, m, shift, S);
    const uint32_t hf = threadIdx.x & 1u;
    for (uint32_t s0 = threadIdx.x >> 1; s0 < m; s0 += PAIRS * PER_PAIR) {
        uint64_t q[PER_PAIR], ra[PER_PAIR], rb[PER_PAIR];
        bool bad[PER_PAIR];
#pragma unroll
        for (int u = 0; u < PER_PAIR; ++u) q[u] = S.q[min(s0 + u * PAIRS, m - 1)];
        rank4_pair_compute<L, PER_PAIR>(lines, super, n, q, hf, ra, rb, bad);
#pragma unroll
        for (int u = 0; u < PER_PAIR; ++u) {
            const uint32_t sl = s0 + u * PAIRS;
            if (sl < m) {
                const uint32_t ti = S.tile_of[sl];
                if (STAGE) {
                    const u64x2_t v = {ra[u], rb[u]};
                    R[2 * ti + hf] = v;
                } else {  // a lone 32-byte row: a plain store, which L2 can merge with its neighbours
                    reinterpret_cast<ulonglong2 *>(out4 + 4 * (base + ti))[hf] = make_ulonglong2(ra[u], rb[u]);
                }
                if (bad[u] && hf == 0) atomicOr(err, 1u);
            }
        }
    }
    if (STAGE) {
        __syncthreads();
        for (uint32_t k = threadIdx.x; k < 2 * m; k += SWEEP_BLOCK) store_once2(out4 + 4 * base + 2 * k, R[k].x, R[k].y);
    }
}

// Geometry of each layout as the host needs it.
struct QrGeom {
    uint64_t data, sb_lines, max_n, super_elem;  // super_elem: bytes per offset (0: no offset array)
};

bool qr_geom(int layout, QrGeom &g) {
    switch (layout) {
        case QR_LAYOUT_16: g = {QR16::DATA, QR16::SB_LINES, QR16::MAX_N, 4}; return true;
        case QR_LAYOUT_32: g = {QR32::DATA, QR32::SB_LINES, QR32::MAX_N, 8}; return true;
        case QR_LAYOUT_16P: g = {QR16P::DATA, QR16P::SB_LINES, QR16P::MAX_N, 4}; return true;
        case QR_LAYOUT_64: g = {QR64::DATA, QR64::SB_LINES, QR64::MAX_N, 0}; return true;
        case QR_LAYOUT_24_8: g = {QR24_8::DATA, QR24_8::SB_LINES, QR24_8::MAX_N, 8}; return true;
        default: return false;
    }
}

// f(L{}) for the layout's trait type.
template <class F>
auto qr_dispatch(int layout, F &&f) {
    switch (layout) {
        case QR_LAYOUT_32: return f(QR32{});
        case QR_LAYOUT_16P: return f(QR16P{});
        case QR_LAYOUT_64: return f(QR64{});
        case QR_LAYOUT_24_8: return f(QR24_8{});
        default: return f(QR16{});
    }
}

uint64_t super_bytes_of(const qr_quadrank_s *h) {
    QrGeom g{};
    return qr_geom(h->layout, g) ? h->n_sb * 4 * g.super_elem : 0;
}

void release(qr_quadrank_s *h) {
    if (!h) return;
    if (h->lines) (void)hipFree(h->lines);
    if (h->super) (void)hipFree(h->super);
    if (h->err) (void)hipFree(h->err);
    delete h;
}

uint64_t grid_for(uint64_t nq, int pl, int block, int grid_waves, int lanes) {
    uint64_t blocks = (lanes * ((nq + pl - 1) / pl) + block - 1) / block;
    if (grid_waves > 0) blocks = std::min<uint64_t>(blocks, std::max<uint64_t>(1, (uint64_t)cu_count() * grid_waves * 64 / block));
    return std::max<uint64_t>(1, std::min<uint64_t>(blocks, 0x7fffffffull));
}

template <class L>
hipError_t build_t(const uint64_t *d_packed2, uint64_t n, uint64_t *lines, void *super, hipStream_t stream) {
    const uint64_t n_lines = n / L::DATA + 1, n_sb = L::SB_LINES ? (n_lines - 1) / L::SB_LINES + 1 : 0;
    const uint64_t n_groups = (n_lines - 1) / GROUP_LINES + 1, n_words = (n + 31) / 32;
    uint32_t *cnt = nullptr;
    uint64_t *base = nullptr;
    if (hipMalloc(&cnt, n_groups * 16) != hipSuccess || hipMalloc(&base, n_groups * 32) != hipSuccess) {
        (void)hipGetLastError();
        if (cnt) (void)hipFree(cnt);
        return hipErrorOutOfMemory;
    }
    hipLaunchKernelGGL(qr_count_kernel<L>, dim3((uint32_t)((n_groups + COUNT_GROUPS - 1) / COUNT_GROUPS)),
                       dim3(64 * COUNT_GROUPS), 0, stream, d_packed2, n, n_words, n_groups, cnt);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        if constexpr (L::SHIFT != 0 && L::SB_LINES == GROUP_LINES) {  // a group is a superblock
            e = launch_scan_counts(cnt, n_groups, 4, L::SHIFT, base, reinterpret_cast<uint32_t *>(super), stream);
        } else {
            e = launch_scan_counts(cnt, n_groups, 4, 0, base, nullptr, stream);
            if (e == hipSuccess && L::ID == QR_LAYOUT_16P) {
                hipLaunchKernelGGL(qr_paired_super_kernel, dim3((uint32_t)((4 * n_sb + 255) / 256)), dim3(256), 0, stream,
                                   base, cnt, n_groups, n_sb, L::SHIFT, reinterpret_cast<uint32_t *>(super));
                e = hipGetLastError();
            } else if (e == hipSuccess && L::SB_LINES != 0) {
                hipLaunchKernelGGL(qr_exact_super_kernel, dim3((uint32_t)((4 * n_sb + 255) / 256)), dim3(256), 0, stream,
                                   base, n_groups, n_sb, (uint64_t)(L::SB_LINES / GROUP_LINES),
                                   reinterpret_cast<uint64_t *>(super));
                e = hipGetLastError();
            }
        }
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(qr_write_kernel<L>, dim3((uint32_t)n_groups), dim3(128), 0, stream, d_packed2, n, n_words, base,
                           reinterpret_cast<const uint32_t *>(super), n_lines, lines);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    (void)hipFree(cnt);
    (void)hipFree(base);
    return e;
}

template <class L, bool PREFIX, int QPT>
void launch_rank1_sweep(qr_quadrank h, const uint64_t *d_q, const uint8_t *d_c, uint64_t nq, uint64_t *d_out,
                        hipStream_t s) {
    const dim3 g((uint32_t)((nq + SWEEP_BLOCK * QPT - 1) / (SWEEP_BLOCK * QPT))), b(SWEEP_BLOCK);
    const uint4 *Ln = reinterpret_cast<const uint4 *>(h->lines);
    const auto *S = reinterpret_cast<const typename L::Super *>(h->super);
    const uint32_t shift = sweep_shift(h->n);
    if (h->tune.per_lane == 2)
        hipLaunchKernelGGL((qr_sym_sweep_kernel<L, 2, PREFIX, QPT>), g, b, 0, s, Ln, S, h->n, d_q, d_c, nq, d_out, h->err,
                           shift);
    else
        hipLaunchKernelGGL((qr_sym_sweep_kernel<L, 1, PREFIX, QPT>), g, b, 0, s, Ln, S, h->n, d_q, d_c, nq, d_out, h->err,
                           shift);
}

template <class L>
void launch_rank4_sweep(qr_quadrank h, const uint64_t *d_q, uint64_t nq, uint64_t *d_out4, hipStream_t s) {
    const uint4 *Ln = reinterpret_cast<const uint4 *>(h->lines);
    const auto *S = reinterpret_cast<const typename L::Super *>(h->super);
    const uint32_t shift = sweep_shift(h->n);
    const int qpt = h->tune.sweep / SWEEP_BLOCK;
    const dim3 g((uint32_t)((nq + h->tune.sweep - 1) / h->tune.sweep)), b(SWEEP_BLOCK);
#define QR_R4S(P, Q) hipLaunchKernelGGL((qr_rank4_sweep_kernel<L, P, Q>), g, b, 0, s, Ln, S, h->n, d_q, nq, d_out4, h->err, shift)
    if (h->tune.per_lane == 2) {
        if (qpt == 4) QR_R4S(2, 4); else if (qpt == 8) QR_R4S(2, 8); else QR_R4S(2, 16);
    } else {
        if (qpt == 4) QR_R4S(1, 4); else if (qpt == 8) QR_R4S(1, 8); else QR_R4S(1, 16);
    }
#undef QR_R4S
}

template <class L, bool PREFIX>
int launch_rank1(qr_quadrank h, const uint64_t *d_q, const uint8_t *d_c, uint64_t nq, uint64_t *d_out, hipStream_t s) {
    if (sweep_fits(h->tune.sweep, nq)) {
        switch (h->tune.sweep / SWEEP_BLOCK) {
            case 4: launch_rank1_sweep<L, PREFIX, 4>(h, d_q, d_c, nq, d_out, s); break;
            case 8: launch_rank1_sweep<L, PREFIX, 8>(h, d_q, d_c, nq, d_out, s); break;
            default: launch_rank1_sweep<L, PREFIX, 16>(h, d_q, d_c, nq, d_out, s); break;
        }
        QR_HIP(hipGetLastError());
        return QR_OK;
    }
    const int block = h->tune.block ? h->tune.block : 256, pl = h->tune.per_lane ? h->tune.per_lane : 1;
    const int lanes = h->tune.lanes == 1 ? 1 : 2;
    const dim3 g((uint32_t)grid_for(nq, pl, block, h->tune.grid_waves, lanes)), b(block);
    const uint4 *Ln = reinterpret_cast<const uint4 *>(h->lines);
    const auto *S = reinterpret_cast<const typename L::Super *>(h->super);
#define QR_RANK1(K, P) hipLaunchKernelGGL((K<L, P>), g, b, 0, s, Ln, S, h->n, d_q, d_c, nq, d_out, h->err)
#define QR_RANK1_PL(K)                          \
    switch (pl) {                               \
        case 1: QR_RANK1(K, 1); break;          \
        case 2: QR_RANK1(K, 2); break;          \
        case 4: QR_RANK1(K, 4); break;          \
        default: QR_RANK1(K, 8); break;         \
    }
    if (PREFIX) {
        if (lanes == 2) {
            QR_RANK1_PL(qr_prefix_pair_kernel)
        } else {
            QR_RANK1_PL(qr_prefix_kernel)
        }
    } else {
        if (lanes == 2) {
            QR_RANK1_PL(qr_rank1_pair_kernel)
        } else {
            QR_RANK1_PL(qr_rank1_kernel)
        }
    }
#undef QR_RANK1_PL
#undef QR_RANK1
    QR_HIP(hipGetLastError());
    return QR_OK;
}

template <class L>
int launch_rank4(qr_quadrank h, const uint64_t *d_q, uint64_t nq, uint64_t *d_out4, hipStream_t s) {
    if (sweep_fits(h->tune.sweep, nq)) {
        launch_rank4_sweep<L>(h, d_q, nq, d_out4, s);
        QR_HIP(hipGetLastError());
        return QR_OK;
    }
    const int block = h->tune.block ? h->tune.block : 256, pl = h->tune.per_lane ? h->tune.per_lane : 1;
    const int lanes = h->tune.lanes == 1 ? 1 : 2;
    const dim3 g((uint32_t)grid_for(nq, pl, block, h->tune.grid_waves, lanes)), b(block);
    const uint4 *Ln = reinterpret_cast<const uint4 *>(h->lines);
    const auto *S = reinterpret_cast<const typename L::Super *>(h->super);
#define QR_RANK4(K, P) hipLaunchKernelGGL((K<L, P>), g, b, 0, s, Ln, S, h->n, d_q, nq, d_out4, h->err)
    if (lanes == 2) {
        switch (pl) {
            case 1: QR_RANK4(qr_rank4_pair_kernel, 1); break;
            case 2: QR_RANK4(qr_rank4_pair_kernel, 2); break;
            case 4: QR_RANK4(qr_rank4_pair_kernel, 4); break;
            default: QR_RANK4(qr_rank4_pair_kernel, 8); break;
        }
    } else {
        switch (pl) {
            case 1: QR_RANK4(qr_rank4_kernel, 1); break;
            case 2: QR_RANK4(qr_rank4_kernel, 2); break;
            case 4: QR_RANK4(qr_rank4_kernel, 4); break;
            default: QR_RANK4(qr_rank4_kernel, 8); break;
        }
    }
#undef QR_RANK4
    QR_HIP(hipGetLastError());
    return QR_OK;
}

}  // namespace

namespace qr {

// Build a QuadRank layout into caller-provided arrays (used by the FM-index build).
int quadrank_build_into(const uint64_t *d_packed2, uint64_t n, int layout, uint64_t *lines, void *super,
                        hipStream_t stream) {
    hipError_t e = qr_dispatch(layout, [&](auto tag) { return build_t<decltype(tag)>(d_packed2, n, lines, super, stream); });
    if (e == hipErrorOutOfMemory) {
        set_error("quadrank build: temporary allocation failed");
        return QR_ENOMEM;
    }
    if (e != hipSuccess) {
        set_error("quadrank build: %s", hipGetErrorString(e));
        return QR_EHIP;
    }
    return QR_OK;
}

}  // namespace qr

extern "C" {

int quadrank_build_ex(const uint64_t *d_packed2, uint64_t n, int layout, hipStream_t stream, qr_quadrank *out) {
    if (!out) {
        set_error("quadrank_build: out is NULL");
        return QR_EINVAL;
    }
    *out = nullptr;
    if (((uintptr_t)d_packed2 & 7) || (!d_packed2 && n)) {
        set_error("quadrank_build: d_packed2 is NULL (with n = %llu) or not 8-byte aligned", (unsigned long long)n);
        return QR_EINVAL;
    }
    QrGeom geo{};
    if (!qr_geom(layout, geo)) {
        set_error("quadrank_build: unknown layout %d", layout);
        return QR_EINVAL;
    }
    const uint64_t max_n = geo.max_n;
    if (n > max_n) {
        set_error("quadrank_build: n = %llu exceeds the layout limit %llu", (unsigned long long)n,
                  (unsigned long long)max_n);
        return QR_ERANGE;
    }
    qr_quadrank_s *h = new (std::nothrow) qr_quadrank_s{};
    if (!h) return QR_ENOMEM;
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return QR_EHIP;
    }
    h->layout = layout;
    h->n = n;
    h->n_lines = n / geo.data + 1;
    h->n_sb = geo.sb_lines ? (h->n_lines - 1) / geo.sb_lines + 1 : 0;
    h->tune = qr_tuning{256, 1, 0, 2, 0};
    const size_t super_bytes = h->n_sb * 4 * geo.super_elem;
    if (hipMalloc(&h->lines, h->n_lines * 128) != hipSuccess ||
        (super_bytes && hipMalloc(&h->super, super_bytes) != hipSuccess) || hipMalloc(&h->err, 4) != hipSuccess) {
        (void)hipGetLastError();
        set_error("quadrank_build: device allocation of %llu bytes failed",
                  (unsigned long long)(h->n_lines * 128 + super_bytes));
        release(h);
        return QR_ENOMEM;
    }
    if (hipMemsetAsync(h->err, 0, 4, stream) != hipSuccess) {
        release(h);
        return QR_EHIP;
    }
    const hipError_t e =
        qr_dispatch(layout, [&](auto tag) { return build_t<decltype(tag)>(d_packed2, n, h->lines, h->super, stream); });
    if (e != hipSuccess) {
        set_error("quadrank_build: %s", hipGetErrorString(e));
        release(h);
        return e == hipErrorOutOfMemory ? QR_ENOMEM : QR_EHIP;
    }
    *out = h;
    return QR_OK;
}

int quadrank_build(const uint64_t *d_packed2, uint64_t n, hipStream_t stream, qr_quadrank *out) {
    return quadrank_build_ex(d_packed2, n, QR_LAYOUT_16, stream, out);
}

// out_align: 8 for u64 outputs, 16 for the rank4 rows (written as 16-byte pairs)
static int qr_launch_common(qr_quadrank h, uint64_t nq, const void *a, const void *b, uintptr_t out_align,
                            const char *what) {
    if (!h || (nq && (!a || !b))) {
        set_error("%s: null handle or pointer", what);
        return QR_EINVAL;
    }
    if (((uintptr_t)a & 7) || ((uintptr_t)b & (out_align - 1))) {
        set_error("%s: d_q must be 8-byte and the output %u-byte aligned", what, (unsigned)out_align);
        return QR_EINVAL;
    }
    return check_device(h->device);
}

int quadrank_rank(qr_quadrank h, const uint64_t *d_q, const uint8_t *d_c, uint64_t nq, uint64_t *d_out,
                  hipStream_t stream) {
    int rc = qr_launch_common(h, nq, d_q, d_out, 8, "quadrank_rank");
    if (rc) return rc;
    if (nq && !d_c) {
        set_error("quadrank_rank: d_c is NULL");
        return QR_EINVAL;
    }
    if (!nq) return QR_OK;
    return qr_dispatch(h->layout, [&](auto tag) { return launch_rank1<decltype(tag), false>(h, d_q, d_c, nq, d_out, stream); });
}

int quadrank_prefix_rank(qr_quadrank h, const uint64_t *d_q, const uint8_t *d_c, uint64_t nq, uint64_t *d_out,
                         hipStream_t stream) {
    int rc = qr_launch_common(h, nq, d_q, d_out, 8, "quadrank_prefix_rank");
    if (rc) return rc;
    if (nq && !d_c) {
        set_error("quadrank_prefix_rank: d_c is NULL");
        return QR_EINVAL;
    }
    if (!nq) return QR_OK;
    return qr_dispatch(h->layout, [&](auto tag) { return launch_rank1<decltype(tag), true>(h, d_q, d_c, nq, d_out, stream); });
}

int quadrank_rank4(qr_quadrank h, const uint64_t *d_q, uint64_t nq, uint64_t *d_out4, hipStream_t stream) {
    int rc = qr_launch_common(h, nq, d_q, d_out4, 16, "quadrank_rank4");
    if (rc) return rc;
    if (!nq) return QR_OK;
    return qr_dispatch(h->layout, [&](auto tag) { return launch_rank4<decltype(tag)>(h, d_q, nq, d_out4, stream); });
}

int quadrank_check(qr_quadrank h, hipStream_t stream) {
    if (!h) return QR_EINVAL;
    int rc = check_device(h->device);
    if (rc) return rc;
    uint32_t v = 0;
    QR_HIP(hipStreamSynchronize(stream));
    QR_HIP(hipMemcpy(&v, h->err, 4, hipMemcpyDeviceToHost));
    QR_HIP(hipMemset(h->err, 0, 4));
    if (v) {
        set_error("quadrank: a query had q > n or a symbol > 3");
        return QR_ERANGE;
    }
    return QR_OK;
}

int quadrank_free(qr_quadrank h) {
    release(h);
    return QR_OK;
}

uint64_t quadrank_len(qr_quadrank h) { return h ? h->n : 0; }
uint64_t quadrank_bytes(qr_quadrank h) {
    return h ? h->n_lines * 128 + super_bytes_of(h) : 0;
}
int quadrank_layout_kind(qr_quadrank h) { return h ? h->layout : -1; }

int quadrank_layout(qr_quadrank h, const void **d_lines, uint64_t *n_lines, const void **d_super,
                    uint64_t *n_super) {
    if (!h) return QR_EINVAL;
    if (d_lines) *d_lines = h->lines;
    if (n_lines) *n_lines = h->n_lines;
    if (d_super) *d_super = h->super;
    if (n_super) *n_super = h->n_sb;
    return QR_OK;
}

int quadrank_export(qr_quadrank h, void *h_lines, void *h_super) {
    if (!h) return QR_EINVAL;
    int rc = check_device(h->device);
    if (rc) return rc;
    if (h_lines) QR_HIP(hipMemcpy(h_lines, h->lines, h->n_lines * 128, hipMemcpyDeviceToHost));
    if (h_super && super_bytes_of(h)) QR_HIP(hipMemcpy(h_super, h->super, super_bytes_of(h), hipMemcpyDeviceToHost));
    return QR_OK;
}

int quadrank_set_tuning(qr_quadrank h, const qr_tuning *t) {
    if (!h || !t) return QR_EINVAL;
    if ((t->block && (t->block < 64 || t->block > 256 || t->block % 64)) ||
        (t->per_lane && t->per_lane != 1 && t->per_lane != 2 && t->per_lane != 4 && t->per_lane != 8) ||
        t->grid_waves < 0 || t->grid_waves > 64 || (t->lanes != 0 && t->lanes != 1 && t->lanes != 2)) {
        set_error("quadrank_set_tuning: block 64..256 step 64, per_lane 1/2/4/8, grid_waves 0..64, lanes 1/2");
        return QR_EINVAL;
    }
    if (!sweep_tuning_ok(t)) {
        set_error("quadrank_set_tuning: sweep must be 0, 1024, 2048 or 4096, with lanes 2 and per_lane 1 or 2");
        return QR_EINVAL;
    }
    h->tune = *t;
    if (!h->tune.lanes) h->tune.lanes = 2;
    return QR_OK;
}

}  // extern "C"
