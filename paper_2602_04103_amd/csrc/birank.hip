// BiRank on gfx950 (paper Section 3): binary rank with a delta inlined in every 128-byte line.
//
// Two layouts, both with the delta measured to the line's middle (line bit 512), so each 64-byte
// half of a line is one half of the block and a query popcounts at most 512 bits (Eq. (1)):
//
//   BR16 (default; the paper's BiRank16 re-derived for 128-byte lines)
//     line j: bits [0,16) b_j, bits [16,1024) input bits [1008 j, 1008 j + 1008)
//     b_j = rank(1008 j + 496) - 2^10 s_{j/64};  s_i = floor(rank(64512 i) / 2^10) (u32, the
//     shifted 32-bit offset of Section 3 with shift 10: 64 lines of 1008 bits fill 16 bits)
//     bounds: b_j <= 63*1008 + 496 + 1023 = 65023 < 2^16; s_i < 2^32 for n < 2^42
//   BR32 (the paper's BiRank32 variant: a 32-bit inline value, much smaller offset array)
//     line j: bits [0,32) b_j, bits [32,1024) input bits [992 j, 992 j + 992)
//     b_j = rank(992 j + 480) - s_{j/2^22};  s_i = rank(992 * 2^22 * i) (u64, exact)
//     bounds: b_j <= (2^22 - 1)*992 + 480 < 2^32; the offset array has one entry per 4.16e9 bits
//   BR16P (BR16 with paired superblocks: one offset per 128 lines, at the pair's middle)
//   BR64 (the paper's BiRank64: an absolute 64-bit rank per line, no offset array)
//   BR16X2 (the paper's BiRank16x2: deltas to line bits 256 and 768, a quarter line counted)
//     the last three are defined, with their bounds, beside their layout traits (birank_dev.hpp)
//
// floor(n/B) + 1 lines, so q = n always has a line; bits past n are stored as zero and every
// delta is taken over that zero-padded text.
//
// Query: j = floor(q/B), p = q - B j + HDR (line bit of q);
//   rank(q) = offset_j + b_j + popcount(line bits [512, p))   if p >= 512
//   rank(q) = offset_j + b_j - popcount(line bits [p, 512))   if p <  512
// (BR16X2 counts between p and its anchor, line bit 256 or 768, with that anchor's delta.)
#include <algorithm>
#include <new>

#include "common.hpp"
#include "birank_dev.hpp"
#include "sweep.hpp"

using namespace qr;

namespace {

constexpr uint32_t GROUP_LINES = 64;  // lines per build workgroup (BR16: one superblock)

}  // namespace

struct qr_birank_s {
    int device;
    int layout;  // QR_LAYOUT_16, _32, _16P, _64 or _16X2
    uint64_t n, n_lines, n_sb;
    uint64_t *lines;  // n_lines * 16 words
    void *super;      // n_sb offsets (u32 for the 16-bit layouts, u64 for the 32-bit one; none for BR64)
    uint32_t *err;    // sticky device error word
    qr_tuning tune;
};

namespace {

__device__ __forceinline__ uint64_t masked_word(const uint64_t *__restrict__ bits, uint64_t w, uint64_t n,
                                                uint64_t n_words) {
    if (w >= n_words) return 0;
    uint64_t x = bits[w];
    uint64_t first = w * 64;
    if (first + 64 > n) x &= (1ull << (n - first)) - 1ull;  // n - first in [1, 63] since w < n_words
    return x;
}

// Pass 1: number of 1 bits in each group of 64 lines (GROUP_LINES * DATA / 64 input words), one
// wavefront per group and COUNT_GROUPS groups per workgroup.  Groups made only of whole words below
// n are read with 16-byte loads when the input is 16-byte aligned (a group is an even number of
// words); the last group, or an input aligned to 8 bytes only, takes the masked word path.
constexpr uint32_t COUNT_GROUPS = 4;

template <class L>
__global__ __launch_bounds__(64 * COUNT_GROUPS) void br_count_kernel(const uint64_t *__restrict__ bits, uint64_t n,
                                                                     uint64_t n_words, uint64_t n_groups,
                                                                     uint32_t *__restrict__ cnt) {
    constexpr uint32_t W = GROUP_LINES * L::DATA / 64;
    static_assert(W % 2 == 0, "a group must be a whole number of 16-byte chunks");
    const uint64_t g = (uint64_t)blockIdx.x * COUNT_GROUPS + threadIdx.x / 64;
    if (g >= n_groups) return;
    const uint32_t lane = __lane_id();
    const uint64_t w0 = g * W;
    uint32_t c = 0;
    if (((uintptr_t)bits & 15) == 0 && w0 + W <= n / 64) {
        const uint4 *v = reinterpret_cast<const uint4 *>(bits + w0);
#pragma unroll 4
        for (uint32_t k = lane; k < W / 2; k += 64) {
            const uint4 x = v[k];
            c += __popc(x.x) + __popc(x.y) + __popc(x.z) + __popc(x.w);
        }
    } else {
        for (uint32_t k = lane; k < W; k += 64) c += __popcll(masked_word(bits, w0 + k, n, n_words));
    }
    c = wave_sum(c);
    if (lane == 0) cnt[g] = c;
}

// Offsets of the 32-bit layout: s_i = exact rank at the first line of superblock i.
__global__ void br32_super_kernel(const uint64_t *__restrict__ base, uint64_t n_groups, uint64_t n_sb,
                                  uint64_t *__restrict__ super) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    constexpr uint64_t GPS = BR32::SB_LINES / GROUP_LINES;
    if (i < n_sb) super[i] = base[std::min(i * GPS, n_groups - 1)];
}

// Offsets of paired superblocks: s'_i = the rank at the start of group 2i + 1 (the pair's middle),
// shifted.  A last pair without its upper group takes the rank after its lower group, whose count
// covers all 64 of its (zero-padded) lines.
__global__ void br_paired_super_kernel(const uint64_t *__restrict__ base, const uint32_t *__restrict__ cnt,
                                       uint64_t n_groups, uint64_t n_sb, uint32_t shift, uint32_t *__restrict__ super) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_sb) return;
    const uint64_t g = 2 * i + 1;
    const uint64_t r = g < n_groups ? base[g] : base[g - 1] + cnt[g - 1];
    super[i] = (uint32_t)(r >> shift);
}

// Pass 3: one 64-lane workgroup per group of 64 lines; lane t forms line 64 g + t.
constexpr int OUT_STRIDE = 17;  // padded LDS row (u64) for the staged lines: avoids bank conflicts

template <class L>
__global__ __launch_bounds__(64) void br_write_kernel(const uint64_t *__restrict__ bits, uint64_t n, uint64_t n_words,
                                                      const uint64_t *__restrict__ base,
                                                      const uint32_t *__restrict__ paired_super, uint64_t n_lines,
                                                      uint64_t *__restrict__ lines) {
    constexpr uint32_t W = GROUP_LINES * L::DATA / 64;
    constexpr uint64_t GPS = L::SB_LINES >= GROUP_LINES ? L::SB_LINES / GROUP_LINES : 1;  // groups per superblock
    // one LDS buffer holds the group's input words, then (after a barrier) the staged output lines
    constexpr uint32_t BUF = (W + 2 > 64 * OUT_STRIDE) ? W + 2 : 64 * OUT_STRIDE;
    __shared__ __align__(16) uint64_t buf[BUF];
    uint64_t *in = buf, *stage = buf;
    const uint64_t g = blockIdx.x;
    const int t = threadIdx.x;
    if (((uintptr_t)bits & 15) == 0 && g * W + W <= n / 64) {  // whole words only: 16-byte loads
        const uint4 *v = reinterpret_cast<const uint4 *>(bits + g * W);
        uint4 *d = reinterpret_cast<uint4 *>(in);
#pragma unroll 4
        for (uint32_t k = t; k < W / 2; k += 64) d[k] = v[k];
        if (t < 2) in[W + t] = 0ull;
    } else {
        for (int k = t; k < (int)W + 2; k += 64) in[k] = k < (int)W ? masked_word(bits, g * W + k, n, n_words) : 0ull;
    }
    __syncthreads();

    auto get64 = [&](uint32_t b) -> uint64_t {  // input bits [b, b+64) of this group
        uint32_t w = b >> 6, sh = b & 63;
        uint64_t lo = in[w];
        return sh ? (lo >> sh) | (in[w + 1] << (64 - sh)) : lo;
    };
    const uint32_t b0 = L::DATA * (uint32_t)t;
    uint64_t o[16];
    o[0] = L::HDR < 64 ? get64(b0) << (L::HDR & 63u) : 0ull;  // the header bits stay zero for now
#pragma unroll
    for (int k = 1; k < 16; ++k) o[k] = get64(b0 + 64u * k - L::HDR);
    // ones before each anchor of the line: line bit 512 (middle), or 256 and 768 (quarter anchors)
    uint32_t c_q1 = 0, c_q2 = 0, c_q3 = 0, c_q4 = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) c_q1 += __popcll(o[k]);
#pragma unroll
    for (int k = 4; k < 8; ++k) c_q2 += __popcll(o[k]);
#pragma unroll
    for (int k = 8; k < 12; ++k) c_q3 += __popcll(o[k]);
#pragma unroll
    for (int k = 12; k < 16; ++k) c_q4 += __popcll(o[k]);
    const uint32_t c_tot = c_q1 + c_q2 + c_q3 + c_q4;
    const uint32_t before = wave_inclusive_scan<uint32_t>(c_tot) - c_tot;
    const uint64_t start = base[g] + before;  // rank at the line's first data bit
    // offset of this line's superblock as the query reconstructs it
    uint64_t off = 0;
    if constexpr (L::ID == QR_LAYOUT_16P) {
        off = ((uint64_t)paired_super[g >> 1] << L::SHIFT) - ((g & 1) ? 0ull : L::BIAS);
    } else if constexpr (L::SB_LINES != 0) {
        const uint64_t sb_base = base[(g / GPS) * GPS];
        off = (sb_base >> L::SHIFT) << L::SHIFT;
    }
    if constexpr (L::QUARTER) {
        const uint64_t d0 = start + c_q1 - off, d1 = start + c_q1 + c_q2 + c_q3 - off;
        o[0] |= d0 | (d1 << 16);
    } else {
        o[0] |= start + c_q1 + c_q2 - off;  // fills the HDR header bits (all 64 of them for BR64)
    }
    __syncthreads();  // every lane has read its input words: the buffer now takes the output
#pragma unroll
    for (int k = 0; k < 16; ++k) stage[t * OUT_STRIDE + k] = o[k];
    __syncthreads();
    const uint64_t l0 = g * GROUP_LINES;
    const uint32_t nl = (uint32_t)std::min<uint64_t>(GROUP_LINES, n_lines - l0);
    uint4 *dst = reinterpret_cast<uint4 *>(lines + l0 * 16);
    for (uint32_t e = t; e < nl * 8; e += 64) {  // 8 uint4 per line, coalesced
        const uint64_t *src = stage + (e >> 3) * OUT_STRIDE + (e & 7) * 2;
        uint64_t a = src[0], b = src[1];
        dst[e] = make_uint4((uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32));
    }
}


// One lane per query: the lane loads the half holding q, plus the line's first word for the delta
// when q lies in the upper half.  PER_LANE independent queries per lane, loads before popcounts.
template <class L, int PER_LANE>
__global__ __launch_bounds__(256) void br_rank_kernel(const uint4 *__restrict__ lines,
                                                      const typename L::Super *__restrict__ super, uint64_t n,
                                                      const uint64_t *__restrict__ Q, uint64_t nq,
                                                      uint64_t *__restrict__ out, uint32_t *__restrict__ err) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i0 < nq; i0 += stride * PER_LANE) {
        uint64_t q[PER_LANE], off[PER_LANE];
        uint32_t p[PER_LANE];
        uint2 hdr[PER_LANE];
        uint32_t h[PER_LANE][16];
        bool bad[PER_LANE];
#pragma unroll
        for (int u = 0; u < PER_LANE; ++u) {
            q[u] = load_once(Q + min(i0 + u * stride, nq - 1));
            bad[u] = q[u] > n;
            if (bad[u]) q[u] = 0;  // line 0 always exists; the output is overwritten below
        }
#pragma unroll
        for (int u = 0; u < PER_LANE; ++u) {
            const uint64_t j = line_of<L>(q[u]);
            p[u] = (uint32_t)(q[u] - j * L::DATA) + L::HDR;
            const bool up = p[u] >= L::MID;
            const uint4 *H = lines + j * 8 + (up ? 4 : 0);
            const uint4 a = H[0], b = H[1], c = H[2], d = H[3];
            h[u][0] = a.x, h[u][1] = a.y, h[u][2] = a.z, h[u][3] = a.w;
            h[u][4] = b.x, h[u][5] = b.y, h[u][6] = b.z, h[u][7] = b.w;
            h[u][8] = c.x, h[u][9] = c.y, h[u][10] = c.z, h[u][11] = c.w;
            h[u][12] = d.x, h[u][13] = d.y, h[u][14] = d.z, h[u][15] = d.w;
            hdr[u] = up ? reinterpret_cast<const uint2 *>(lines)[j * 16] : make_uint2(a.x, a.y);
            off[u] = L::offset(super, j);
        }
        uint64_t r[PER_LANE];
#pragma unroll
        for (int u = 0; u < PER_LANE; ++u) {
            const bool up = p[u] >= L::MID;
            bool fwd;
            const uint32_t cnt = br_count<L>(h[u], up ? p[u] - L::MID : p[u], up, fwd);
            const uint64_t j = line_of<L>(q[u]);
            const uint64_t anchor = off[u] + L::delta(hdr[u].x, hdr[u].y, up, j);
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

// Lane-pair query kernel: lanes 2k and 2k+1 serve the same query; lane h loads half h (64 bytes)
// of the line, so every load instruction of a wave touches 32 lines with 64 contiguous bytes
// each (measured on MI355X: far fewer address-translation misses on multi-GiB structures than one
// lane issuing four loads).  The lane holding the half that contains q popcounts it; lane 0 adds
// the superblock offset and delta; the two contributions are summed across the pair.
// rank(q[u]) for one query per unroll slot u, valid in both lanes of the pair; bad[u] marks q > n.
template <class L, int PER_PAIR>
__device__ __forceinline__ void br_pair_compute(const uint4 *__restrict__ lines,
                                                const typename L::Super *__restrict__ super, uint64_t n,
                                                const uint64_t (&q)[PER_PAIR], uint32_t hf, uint64_t (&r)[PER_PAIR],
                                                bool (&bad)[PER_PAIR]) {
    uint64_t off[PER_PAIR], jj[PER_PAIR];
    uint32_t p[PER_PAIR];
    uint32_t h[PER_PAIR][16];
    // this lane's half line and the superblock offset
#pragma unroll
    for (int u = 0; u < PER_PAIR; ++u) {
        bad[u] = q[u] > n;
        const uint64_t qq = bad[u] ? 0 : q[u];
        const uint64_t j = line_of<L>(qq);
        p[u] = (uint32_t)(qq - j * L::DATA) + L::HDR;
        const uint4 *H = lines + j * 8 + hf * 4;
        const uint4 a = H[0], b = H[1], c = H[2], d = H[3];
        h[u][0] = a.x, h[u][1] = a.y, h[u][2] = a.z, h[u][3] = a.w;
        h[u][4] = b.x, h[u][5] = b.y, h[u][6] = b.z, h[u][7] = b.w;
        h[u][8] = c.x, h[u][9] = c.y, h[u][10] = c.z, h[u][11] = c.w;
        h[u][12] = d.x, h[u][13] = d.y, h[u][14] = d.z, h[u][15] = d.w;
        off[u] = L::offset(super, j);
        jj[u] = j;
    }
    // count and combine across the pair: the lane holding q's half adds or subtracts its count,
    // lane 0 (which holds the header) adds the anchor's rank
#pragma unroll
    for (int u = 0; u < PER_PAIR; ++u) {
        const bool up = p[u] >= L::MID;
        bool fwd;
        const uint32_t cnt = br_count<L>(h[u], up ? p[u] - L::MID : p[u], up, fwd) & (((uint32_t)up == hf) ? ~0u : 0u);
        uint64_t mine = fwd ? (uint64_t)cnt : 0ull - (uint64_t)cnt;
        if (hf == 0) mine += off[u] + L::delta(h[u][0], h[u][1], up, jj[u]);
        r[u] = bad[u] ? ~0ull : mine + pair_swap64(mine);
    }
}

template <class L, int PER_PAIR>
__global__ __launch_bounds__(256) void br_rank_pair_kernel(const uint4 *__restrict__ lines,
                                                           const typename L::Super *__restrict__ super, uint64_t n,
                                                           const uint64_t *__restrict__ Q, uint64_t nq,
                                                           uint64_t *__restrict__ out, uint32_t *__restrict__ err) {
    const uint32_t hf = threadIdx.x & 1u;
    const uint64_t pairs = ((uint64_t)gridDim.x * blockDim.x) >> 1;
    for (uint64_t i0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 1; i0 < nq; i0 += pairs * PER_PAIR) {
        uint64_t q[PER_PAIR], r[PER_PAIR];
        bool bad[PER_PAIR];
        // query positions (index clamped so every load is unconditional and in bounds)
#pragma unroll
        for (int u = 0; u < PER_PAIR; ++u) q[u] = load_once(Q + min(i0 + u * pairs, nq - 1));
        br_pair_compute<L, PER_PAIR>(lines, super, n, q, hf, r, bad);
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
template <class L, int PER_PAIR, int QPT>
__global__ __launch_bounds__(SWEEP_BLOCK) void br_rank_sweep_kernel(const uint4 *__restrict__ lines,
                                                                    const typename L::Super *__restrict__ super,
                                                                    uint64_t n, const uint64_t *__restrict__ Q,
                                                                    uint64_t nq, uint64_t *__restrict__ out,
                                                                    uint32_t *__restrict__ err, uint32_t shift) {
    __shared__ SweepLds<QPT, false> S;
    constexpr uint32_t PAIRS = SWEEP_BLOCK / 2;
    const uint64_t base = (uint64_t)blockIdx.x * (SWEEP_BLOCK * QPT);
    const uint32_t m = (uint32_t)min<uint64_t>(SWEEP_BLOCK * QPT, nq - base);
    sweep_sort<QPT, false>(Q, nullptr, base, m, shift, S);
    const uint32_t hf = threadIdx.x & 1u;
    for (uint32_t s0 = threadIdx.x >> 1; s0 < m; s0 += PAIRS * PER_PAIR) {
        uint64_t q[PER_PAIR], r[PER_PAIR];
        bool bad[PER_PAIR];
#pragma unroll
        for (int u = 0; u < PER_PAIR; ++u) q[u] = S.q[min(s0 + u * PAIRS, m - 1)];  // past m: discarded
        br_pair_compute<L, PER_PAIR>(lines, super, n, q, hf, r, bad);
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
    sweep_store<QPT, false>(out, base, m, S);
}

template <class L, int PL>
hipError_t launch_rank_t(const qr_birank_s *h, const uint64_t *d_q, uint64_t nq, uint64_t *d_out, hipStream_t s) {
    const int block = h->tune.block ? h->tune.block : 256;
    const int lanes = h->tune.lanes == 1 ? 1 : 2;
    uint64_t blocks = (lanes * ((nq + PL - 1) / PL) + block - 1) / block;
    if (h->tune.grid_waves > 0)
        blocks = std::min<uint64_t>(blocks, std::max<uint64_t>(1, (uint64_t)cu_count() * h->tune.grid_waves * 64 / block));
    blocks = std::max<uint64_t>(1, std::min<uint64_t>(blocks, 0x7fffffffull));
    const uint4 *L4 = reinterpret_cast<const uint4 *>(h->lines);
    const auto *S = reinterpret_cast<const typename L::Super *>(h->super);
    if (lanes == 2)
        hipLaunchKernelGGL((br_rank_pair_kernel<L, PL>), dim3((uint32_t)blocks), dim3(block), 0, s, L4, S, h->n, d_q, nq,
                           d_out, h->err);
    else
        hipLaunchKernelGGL((br_rank_kernel<L, PL>), dim3((uint32_t)blocks), dim3(block), 0, s, L4, S, h->n, d_q, nq,
                           d_out, h->err);
    return hipGetLastError();
}

template <class L, int PL, int QPT>
hipError_t launch_rank_sweep(const qr_birank_s *h, const uint64_t *d_q, uint64_t nq, uint64_t *d_out, hipStream_t s) {
    const dim3 g((uint32_t)((nq + SWEEP_BLOCK * QPT - 1) / (SWEEP_BLOCK * QPT))), b(SWEEP_BLOCK);
    const uint4 *L4 = reinterpret_cast<const uint4 *>(h->lines);
    const auto *S = reinterpret_cast<const typename L::Super *>(h->super);
    hipLaunchKernelGGL((br_rank_sweep_kernel<L, PL, QPT>), g, b, 0, s, L4, S, h->n, d_q, nq, d_out, h->err,
                       sweep_shift(h->n));
    return hipGetLastError();
}

template <class L>
hipError_t launch_rank(const qr_birank_s *h, const uint64_t *d_q, uint64_t nq, uint64_t *d_out, hipStream_t s) {
    if (sweep_fits(h->tune.sweep, nq)) {
        const bool two = h->tune.per_lane == 2;
        switch (h->tune.sweep / SWEEP_BLOCK) {
            case 4: return two ? launch_rank_sweep<L, 2, 4>(h, d_q, nq, d_out, s) : launch_rank_sweep<L, 1, 4>(h, d_q, nq, d_out, s);
            case 8: return two ? launch_rank_sweep<L, 2, 8>(h, d_q, nq, d_out, s) : launch_rank_sweep<L, 1, 8>(h, d_q, nq, d_out, s);
            default: return two ? launch_rank_sweep<L, 2, 16>(h, d_q, nq, d_out, s) : launch_rank_sweep<L, 1, 16>(h, d_q, nq, d_out, s);
        }
    }
    switch (h->tune.per_lane ? h->tune.per_lane : 1) {
        case 1: return launch_rank_t<L, 1>(h, d_q, nq, d_out, s);
        case 2: return launch_rank_t<L, 2>(h, d_q, nq, d_out, s);
        case 4: return launch_rank_t<L, 4>(h, d_q, nq, d_out, s);
        default: return launch_rank_t<L, 8>(h, d_q, nq, d_out, s);
    }
}

template <class L>
hipError_t build_t(qr_birank_s *h, const uint64_t *d_bits, uint32_t *cnt, uint64_t *base, uint64_t n_groups,
                   hipStream_t stream) {
    const uint64_t n_words = (h->n + 63) / 64;
    hipLaunchKernelGGL(br_count_kernel<L>, dim3((uint32_t)((n_groups + COUNT_GROUPS - 1) / COUNT_GROUPS)),
                       dim3(64 * COUNT_GROUPS), 0, stream, d_bits, h->n, n_words, n_groups, cnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if constexpr (L::SHIFT != 0 && L::SB_LINES == GROUP_LINES) {
        // a group is a superblock: the scan writes the shifted offsets
        e = launch_scan_counts(cnt, n_groups, 1, L::SHIFT, base, reinterpret_cast<uint32_t *>(h->super), stream);
    } else {  // scan into base, then the offsets of the layout (none for BR64)
        e = launch_scan_counts(cnt, n_groups, 1, 0, base, nullptr, stream);
        if (e == hipSuccess && L::ID == QR_LAYOUT_32) {
            hipLaunchKernelGGL(br32_super_kernel, dim3((uint32_t)((h->n_sb + 255) / 256)), dim3(256), 0, stream, base,
                               n_groups, h->n_sb, reinterpret_cast<uint64_t *>(h->super));
            e = hipGetLastError();
        } else if (e == hipSuccess && L::ID == QR_LAYOUT_16P) {
            hipLaunchKernelGGL(br_paired_super_kernel, dim3((uint32_t)((h->n_sb + 255) / 256)), dim3(256), 0, stream, base,
                               cnt, n_groups, h->n_sb, L::SHIFT, reinterpret_cast<uint32_t *>(h->super));
            e = hipGetLastError();
        }
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(br_write_kernel<L>, dim3((uint32_t)n_groups), dim3(64), 0, stream, d_bits, h->n, n_words, base,
                       reinterpret_cast<const uint32_t *>(h->super), h->n_lines, h->lines);
    return hipGetLastError();
}

// Geometry of each layout as the host needs it.
struct BrGeom {
    uint64_t data, sb_lines, max_n, super_elem;  // super_elem: bytes per offset (0: no offset array)
};

bool br_geom(int layout, BrGeom &g) {
    switch (layout) {
        case QR_LAYOUT_16: g = {BR16::DATA, BR16::SB_LINES, BR16::MAX_N, 4}; return true;
        case QR_LAYOUT_32: g = {BR32::DATA, BR32::SB_LINES, BR32::MAX_N, 8}; return true;
        case QR_LAYOUT_16P: g = {BR16P::DATA, BR16P::SB_LINES, BR16P::MAX_N, 4}; return true;
        case QR_LAYOUT_64: g = {BR64::DATA, BR64::SB_LINES, BR64::MAX_N, 0}; return true;
        case QR_LAYOUT_16X2: g = {BR16X2::DATA, BR16X2::SB_LINES, BR16X2::MAX_N, 4}; return true;
        default: return false;
    }
}

// f(L{}) for the layout's trait type.
template <class F>
hipError_t br_dispatch(int layout, F &&f) {
    switch (layout) {
        case QR_LAYOUT_32: return f(BR32{});
        case QR_LAYOUT_16P: return f(BR16P{});
        case QR_LAYOUT_64: return f(BR64{});
        case QR_LAYOUT_16X2: return f(BR16X2{});
        default: return f(BR16{});
    }
}

uint64_t super_bytes_of(const qr_birank_s *h) {
    BrGeom g{};
    return br_geom(h->layout, g) ? h->n_sb * g.super_elem : 0;
}

void release(qr_birank_s *h) {
    if (!h) return;
    if (h->lines) (void)hipFree(h->lines);
    if (h->super) (void)hipFree(h->super);
    if (h->err) (void)hipFree(h->err);
    delete h;
}

}  // namespace

extern "C" {

int birank_build_ex(const uint64_t *d_bits, uint64_t n, int layout, hipStream_t stream, qr_birank *out) {
    if (!out) {
        set_error("birank_build: out is NULL");
        return QR_EINVAL;
    }
    *out = nullptr;
    if (((uintptr_t)d_bits & 7) || (!d_bits && n)) {
        set_error("birank_build: d_bits is NULL (with n = %llu) or not 8-byte aligned", (unsigned long long)n);
        return QR_EINVAL;
    }
    BrGeom geo{};
    if (!br_geom(layout, geo)) {
        set_error("birank_build: unknown layout %d", layout);
        return QR_EINVAL;
    }
    const uint64_t max_n = geo.max_n;
    if (n > max_n) {
        set_error("birank_build: n = %llu exceeds the layout limit %llu", (unsigned long long)n,
                  (unsigned long long)max_n);
        return QR_ERANGE;
    }
    qr_birank_s *h = new (std::nothrow) qr_birank_s{};
    if (!h) return QR_ENOMEM;
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        set_error("hipGetDevice failed");
        return QR_EHIP;
    }
    h->layout = layout;
    h->n = n;
    h->n_lines = n / geo.data + 1;
    h->n_sb = geo.sb_lines ? (h->n_lines - 1) / geo.sb_lines + 1 : 0;
    h->tune = qr_tuning{256, 1, 0, 2, 0};
    const uint64_t n_groups = (h->n_lines - 1) / GROUP_LINES + 1;
    uint32_t *cnt = nullptr;
    uint64_t *base = nullptr;
    auto fail = [&](int code) {
        if (cnt) (void)hipFree(cnt);
        if (base) (void)hipFree(base);
        release(h);
        return code;
    };
    const size_t super_bytes = h->n_sb * geo.super_elem;
    if (hipMalloc(&h->lines, h->n_lines * 128) != hipSuccess ||
        (super_bytes && hipMalloc(&h->super, super_bytes) != hipSuccess) ||
        hipMalloc(&h->err, 4) != hipSuccess || hipMalloc(&cnt, n_groups * 4) != hipSuccess ||
        hipMalloc(&base, n_groups * 8) != hipSuccess) {
        (void)hipGetLastError();
        set_error("birank_build: device allocation of %llu bytes failed",
                  (unsigned long long)(h->n_lines * 128 + super_bytes));
        return fail(QR_ENOMEM);
    }
    if (hipMemsetAsync(h->err, 0, 4, stream) != hipSuccess) return fail(QR_EHIP);
    hipError_t e = br_dispatch(layout, [&](auto tag) { return build_t<decltype(tag)>(h, d_bits, cnt, base, n_groups, stream); });
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        set_error("birank_build: %s", hipGetErrorString(e));
        return fail(QR_EHIP);
    }
    (void)hipFree(cnt);
    (void)hipFree(base);
    *out = h;
    return QR_OK;
}

int birank_build(const uint64_t *d_bits, uint64_t n, hipStream_t stream, qr_birank *out) {
    return birank_build_ex(d_bits, n, QR_LAYOUT_16, stream, out);
}

int birank_rank(qr_birank h, const uint64_t *d_q, uint64_t nq, uint64_t *d_out, hipStream_t stream) {
    if (!h || (nq && (!d_q || !d_out))) {
        set_error("birank_rank: null handle or pointer");
        return QR_EINVAL;
    }
    if (((uintptr_t)d_q & 7) || ((uintptr_t)d_out & 7)) {
        set_error("birank_rank: d_q and d_out must be 8-byte aligned");
        return QR_EINVAL;
    }
    int rc = check_device(h->device);
    if (rc) return rc;
    if (!nq) return QR_OK;
    const hipError_t e =
        br_dispatch(h->layout, [&](auto tag) { return launch_rank<decltype(tag)>(h, d_q, nq, d_out, stream); });
    if (e != hipSuccess) {
        set_error("birank_rank launch: %s", hipGetErrorString(e));
        return QR_EHIP;
    }
    return QR_OK;
}

int birank_check(qr_birank h, hipStream_t stream) {
    if (!h) return QR_EINVAL;
    int rc = check_device(h->device);
    if (rc) return rc;
    uint32_t v = 0;
    QR_HIP(hipStreamSynchronize(stream));
    QR_HIP(hipMemcpy(&v, h->err, 4, hipMemcpyDeviceToHost));
    QR_HIP(hipMemset(h->err, 0, 4));
    if (v) {
        set_error("birank: a query position exceeded n");
        return QR_ERANGE;
    }
    return QR_OK;
}

int birank_free(qr_birank h) {
    if (!h) return QR_OK;
    release(h);
    return QR_OK;
}

uint64_t birank_len(qr_birank h) { return h ? h->n : 0; }
uint64_t birank_bytes(qr_birank h) {
    return h ? h->n_lines * 128 + super_bytes_of(h) : 0;
}
int birank_layout_kind(qr_birank h) { return h ? h->layout : -1; }

int birank_layout(qr_birank h, const void **d_lines, uint64_t *n_lines, const void **d_super, uint64_t *n_super) {
    if (!h) return QR_EINVAL;
    if (d_lines) *d_lines = h->lines;
    if (n_lines) *n_lines = h->n_lines;
    if (d_super) *d_super = h->super;
    if (n_super) *n_super = h->n_sb;
    return QR_OK;
}

int birank_export(qr_birank h, void *h_lines, void *h_super) {
    if (!h) return QR_EINVAL;
    int rc = check_device(h->device);
    if (rc) return rc;
    if (h_lines) QR_HIP(hipMemcpy(h_lines, h->lines, h->n_lines * 128, hipMemcpyDeviceToHost));
    if (h_super && super_bytes_of(h)) QR_HIP(hipMemcpy(h_super, h->super, super_bytes_of(h), hipMemcpyDeviceToHost));
    return QR_OK;
}

int birank_set_tuning(qr_birank h, const qr_tuning *t) {
    if (!h || !t) return QR_EINVAL;
    if (t->block && (t->block < 64 || t->block > 256 || t->block % 64)) {
        set_error("tuning: block must be 64..256 in steps of 64");
        return QR_EINVAL;
    }
    if (t->per_lane && t->per_lane != 1 && t->per_lane != 2 && t->per_lane != 4 && t->per_lane != 8) {
        set_error("tuning: per_lane must be 1, 2, 4 or 8");
        return QR_EINVAL;
    }
    if (t->grid_waves < 0 || t->grid_waves > 64) {
        set_error("tuning: grid_waves must be 0..64");
        return QR_EINVAL;
    }
    if (t->lanes != 0 && t->lanes != 1 && t->lanes != 2) {
        set_error("tuning: lanes must be 1 or 2");
        return QR_EINVAL;
    }
    if (!sweep_tuning_ok(t)) {
        set_error("tuning: sweep must be 0, 1024, 2048 or 4096, with lanes 2 and per_lane 1 or 2");
        return QR_EINVAL;
    }
    h->tune = *t;
    if (!h->tune.lanes) h->tune.lanes = 2;
    return QR_OK;
}

}  // extern "C"
