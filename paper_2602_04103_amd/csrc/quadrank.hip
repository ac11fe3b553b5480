// QuadRank on gfx950 (paper Section 4): DNA rank with four 16-bit deltas inlined per 128-byte line
// and the text stored transposed (a plane of low bits and a plane of high bits).
//
// Line j = 16 little-endian u64 words = 8 pairs (lo_k, hi_k) = (word 2k, word 2k+1), k = 0..7.
// Pair k holds line base slots [64k, 64k+64): bit b of lo_k / hi_k is the low / high bit of slot
// 64k + b.  Slots [0, 32) hold the deltas instead of bases:
//   lo_0 bits [0,16) = b_{j,A}, [16,32) = b_{j,C};   hi_0 bits [0,16) = b_{j,G}, [16,32) = b_{j,T}
// Slots [32, 512) hold bases 480 j .. 480 j + 479 (slot = base - 480 j + 32).
// The line's middle is slot 256 (base 480 j + 224); each half line (pairs 0-3 or 4-7) is one
// 64-byte segment.  b_{j,c} = rank(480 j + 224, c) - 2^12 * s_{j/128, c}.
// Superblock i = lines [128 i, 128 i + 128) = 61440 bases = exactly 1920 packed input words;
//   s_{i,c} = floor(rank(61440 i, c) / 2^12), stored as four u32 per superblock.
// Bound: b <= 127*480 + 224 + (2^12 - 1) = 65279 < 2^16; s < 2^32 for n < 2^44.
// floor(n/480) + 1 lines and floor(n/61440) + 1 superblocks; bases past n are stored as A (code 0)
// and every delta is taken over that padded text, so the padding cancels for every q <= n.
//
// Query: j = floor(q/480), p = q - 480 j + 32 (slot of q);
//   rank(q,c) = 2^12 s_{j/128,c} + b_{j,c} + #c in slots [256, p)   if p >= 256
//   rank(q,c) = 2^12 s_{j/128,c} + b_{j,c} - #c in slots [p, 256)   if p <  256
// Symbol c matches where (lo XNOR c_0) AND (hi XNOR c_1).  rank4 counts the range once per
// plane: T = |lo&hi|, C = |lo| - T, G = |hi| - T, A = len - T - C - G.
#include <algorithm>
#include <new>

#include "common.hpp"
#include "quadrank_dev.hpp"

using namespace qr;

struct qr_quadrank_s {
    int device;
    uint64_t n, n_lines, n_sb;
    uint64_t *lines;  // n_lines * 16 words
    uint32_t *super;  // n_sb * 4
    uint32_t *err;
    qr_tuning tune;
};

namespace {

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

// Pass 1: symbol counts of each superblock (1920 packed words, padded with A).
__global__ __launch_bounds__(256) void qr_count_kernel(const uint64_t *__restrict__ packed, uint64_t n,
                                                       uint64_t n_words, uint32_t *__restrict__ cnt) {
    constexpr uint32_t W = QR_SB_BASES / 32;
    const uint64_t sb = blockIdx.x;
    uint32_t cC = 0, cG = 0, cT = 0;
    for (uint32_t k = threadIdx.x; k < W; k += 256) word_counts(masked_packed(packed, sb * W + k, n, n_words), cC, cG, cT);
    cC = wave_sum(cC), cG = wave_sum(cG), cT = wave_sum(cT);
    __shared__ uint32_t part[4][3];
    if (__lane_id() == 0) part[threadIdx.x / 64][0] = cC, part[threadIdx.x / 64][1] = cG, part[threadIdx.x / 64][2] = cT;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t C = 0, G = 0, T = 0;
        for (int w = 0; w < 4; ++w) C += part[w][0], G += part[w][1], T += part[w][2];
        cnt[4 * sb + 0] = (uint32_t)QR_SB_BASES - C - G - T;
        cnt[4 * sb + 1] = C;
        cnt[4 * sb + 2] = G;
        cnt[4 * sb + 3] = T;
    }
}

// Pass 3: one 128-lane workgroup per superblock; lane t forms line 128 i + t from packed words
// [15 t, 15 t + 15) of the superblock.
constexpr int OUT_STRIDE = 17;

__global__ __launch_bounds__(128) void qr_write_kernel(const uint64_t *__restrict__ packed, uint64_t n,
                                                       uint64_t n_words, const uint64_t *__restrict__ base,
                                                       uint64_t n_lines, uint64_t *__restrict__ lines) {
    constexpr uint32_t W = QR_SB_BASES / 32;  // 1920
    __shared__ uint64_t in[W];
    __shared__ uint64_t stage[128 * OUT_STRIDE];
    __shared__ uint64_t wave_tot[2];
    const uint64_t sb = blockIdx.x;
    const int t = threadIdx.x;
    for (uint32_t k = t; k < W; k += 128) in[k] = masked_packed(packed, sb * W + k, n, n_words);
    __syncthreads();

    uint32_t lo[15], hi[15];
    uint32_t fC = 0, fG = 0, fT = 0, aC = 0, aG = 0, aT = 0;  // first-half and whole-line counts
#pragma unroll
    for (int k = 0; k < 15; ++k) {
        const uint64_t x = in[15 * t + k];
        lo[k] = even_bits(x);
        hi[k] = even_bits(x >> 1);
        if (k < 7) word_counts(x, fC, fG, fT);
        word_counts(x, aC, aG, aT);
    }
    const uint32_t fA = 224 - fC - fG - fT, aA = 480 - aC - aG - aT;
    // Exclusive scan of the four line totals over the 128 lines; each fits 16 bits (<= 61440), so
    // the four are packed into one u64 and scanned together.
    const uint64_t tot = (uint64_t)aA | ((uint64_t)aC << 16) | ((uint64_t)aG << 32) | ((uint64_t)aT << 48);
    uint64_t incl = wave_inclusive_scan<uint64_t>(tot);
    if (__lane_id() == 63) wave_tot[t / 64] = incl;
    __syncthreads();
    if (t >= 64) incl += wave_tot[0];
    const uint64_t before = incl - tot;
    const uint64_t *bs = base + 4 * sb;
    const uint32_t m = (1u << QR_SHIFT) - 1u;
    const uint32_t dA = (uint32_t)(bs[0] & m) + (uint32_t)(before & 0xffff) + fA;
    const uint32_t dC = (uint32_t)(bs[1] & m) + (uint32_t)((before >> 16) & 0xffff) + fC;
    const uint32_t dG = (uint32_t)(bs[2] & m) + (uint32_t)((before >> 32) & 0xffff) + fG;
    const uint32_t dT = (uint32_t)(bs[3] & m) + (uint32_t)((before >> 48) & 0xffff) + fT;

    uint64_t o[16];
    o[0] = (uint64_t)(dA | (dC << 16)) | ((uint64_t)lo[0] << 32);
    o[1] = (uint64_t)(dG | (dT << 16)) | ((uint64_t)hi[0] << 32);
#pragma unroll
    for (int k = 1; k < 8; ++k) {
        o[2 * k] = (uint64_t)lo[2 * k - 1] | ((uint64_t)lo[2 * k] << 32);
        o[2 * k + 1] = (uint64_t)hi[2 * k - 1] | ((uint64_t)hi[2 * k] << 32);
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) stage[t * OUT_STRIDE + k] = o[k];
    __syncthreads();
    const uint64_t l0 = sb * QR_LINES_PER_SB;
    const uint32_t nl = (uint32_t)std::min<uint64_t>(QR_LINES_PER_SB, n_lines - l0);
    uint4 *dst = reinterpret_cast<uint4 *>(lines + l0 * 16);
    for (uint32_t e = t; e < nl * 8; e += 128) {
        const uint64_t *src = stage + (e >> 3) * OUT_STRIDE + (e & 7) * 2;
        uint64_t a = src[0], b = src[1];
        dst[e] = make_uint4((uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32));
    }
}

template <int PER_LANE>
__global__ __launch_bounds__(256) void qr_rank1_kernel(const uint4 *__restrict__ lines, const uint32_t *__restrict__ super,
                                                       uint64_t n, const uint64_t *__restrict__ Q,
                                                       const uint8_t *__restrict__ Cs, uint64_t nq,
                                                       uint64_t *__restrict__ out, uint32_t *__restrict__ err) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i0 < nq; i0 += stride * PER_LANE) {
        uint64_t q[PER_LANE];
        uint32_t c[PER_LANE];
        bool bad[PER_LANE];
        HalfLine hl[PER_LANE];
#pragma unroll
        for (int u = 0; u < PER_LANE; ++u) {
            const uint64_t i = i0 + u * stride;
            q[u] = i < nq ? Q[i] : 0;
            c[u] = i < nq ? Cs[i] : 0;
            bad[u] = q[u] > n || c[u] > 3;
            if (bad[u]) q[u] = 0, c[u] = 0;
        }
#pragma unroll
        for (int u = 0; u < PER_LANE; ++u) load_half(lines, super, q[u], hl[u]);
#pragma unroll
        for (int u = 0; u < PER_LANE; ++u) {
            const uint64_t i = i0 + u * stride;
            if (i >= nq) continue;
            uint64_t r = rank1_from_half(hl[u], c[u]);
            if (bad[u]) {
                r = ~0ull;
                atomicOr(err, 1u);
            }
            out[i] = r;
        }
    }
}

template <int PER_LANE>
__global__ __launch_bounds__(256) void qr_rank4_kernel(const uint4 *__restrict__ lines, const uint32_t *__restrict__ super,
                                                       uint64_t n, const uint64_t *__restrict__ Q, uint64_t nq,
                                                       uint64_t *__restrict__ out4, uint32_t *__restrict__ err) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i0 < nq; i0 += stride * PER_LANE) {
        uint64_t q[PER_LANE];
        bool bad[PER_LANE];
        HalfLine hl[PER_LANE];
#pragma unroll
        for (int u = 0; u < PER_LANE; ++u) {
            const uint64_t i = i0 + u * stride;
            q[u] = i < nq ? Q[i] : 0;
            bad[u] = q[u] > n;
            if (bad[u]) q[u] = 0;
        }
#pragma unroll
        for (int u = 0; u < PER_LANE; ++u) load_half(lines, super, q[u], hl[u]);
#pragma unroll
        for (int u = 0; u < PER_LANE; ++u) {
            const uint64_t i = i0 + u * stride;
            if (i >= nq) continue;
            uint64_t r[4];
            rank4_from_half(hl[u], r);
            if (bad[u]) {
                r[0] = r[1] = r[2] = r[3] = ~0ull;
                atomicOr(err, 1u);
            }
            ulonglong2 *o = reinterpret_cast<ulonglong2 *>(out4 + 4 * i);
            o[0] = make_ulonglong2(r[0], r[1]);
            o[1] = make_ulonglong2(r[2], r[3]);
        }
    }
}

// Lane-pair kernels (default): lanes 2k, 2k+1 serve one query, lane hf loading half hf of the line
// (64 contiguous bytes), so each wave load instruction touches 32 lines.  The lane holding q's half
// counts; lane 0 adds offset and delta; the two contributions are summed across the pair.
template <int PER_PAIR>
__global__ __launch_bounds__(256) void qr_rank1_pair_kernel(const uint4 *__restrict__ lines,
                                                            const uint32_t *__restrict__ super, uint64_t n,
                                                            const uint64_t *__restrict__ Q,
                                                            const uint8_t *__restrict__ Cs, uint64_t nq,
                                                            uint64_t *__restrict__ out, uint32_t *__restrict__ err) {
    const uint32_t hf = threadIdx.x & 1u;
    const uint64_t pairs = ((uint64_t)gridDim.x * blockDim.x) >> 1;
    for (uint64_t i0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 1; i0 < nq; i0 += pairs * PER_PAIR) {
        uint64_t q[PER_PAIR], r[PER_PAIR];
        uint32_t c[PER_PAIR];
        uint4 s[PER_PAIR];
        bool bad[PER_PAIR];
        PairHalf ph[PER_PAIR];
#pragma unroll
        for (int u = 0; u < PER_PAIR; ++u) {
            const uint64_t i = min(i0 + u * pairs, nq - 1);
            q[u] = Q[i];
            c[u] = Cs[i];
        }
#pragma unroll
        for (int u = 0; u < PER_PAIR; ++u) {
            bad[u] = q[u] > n || c[u] > 3;
            load_pair_half(lines, bad[u] ? 0 : q[u], hf, ph[u]);
            s[u] = reinterpret_cast<const uint4 *>(super)[ph[u].j / QR_LINES_PER_SB];
        }
#pragma unroll
        for (int u = 0; u < PER_PAIR; ++u) {
            const uint32_t cc = c[u] & 3u;
            const uint32_t cnt = pair_count1(ph[u], hf, cc);
            const uint64_t mine = hf == 0 ? ((uint64_t)sel4(s[u], cc) << QR_SHIFT) + pair_delta(ph[u], cc) - cnt : (uint64_t)cnt;
            r[u] = bad[u] ? ~0ull : mine + pair_swap64(mine);
        }
#pragma unroll
        for (int u = 0; u < PER_PAIR; ++u) {
            const uint64_t i = i0 + u * pairs;
            if (hf == 0 && i < nq) {
                out[i] = r[u];
                if (bad[u]) atomicOr(err, 1u);
            }
        }
    }
}

template <int PER_PAIR>
__global__ __launch_bounds__(256) void qr_rank4_pair_kernel(const uint4 *__restrict__ lines,
                                                            const uint32_t *__restrict__ super, uint64_t n,
                                                            const uint64_t *__restrict__ Q, uint64_t nq,
                                                            uint64_t *__restrict__ out4, uint32_t *__restrict__ err) {
    const uint32_t hf = threadIdx.x & 1u;
    const uint64_t pairs = ((uint64_t)gridDim.x * blockDim.x) >> 1;
    for (uint64_t i0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 1; i0 < nq; i0 += pairs * PER_PAIR) {
        uint64_t q[PER_PAIR], ra[PER_PAIR], rb[PER_PAIR];
        uint4 s[PER_PAIR];
        bool bad[PER_PAIR];
        PairHalf ph[PER_PAIR];
#pragma unroll
        for (int u = 0; u < PER_PAIR; ++u) q[u] = Q[min(i0 + u * pairs, nq - 1)];
#pragma unroll
        for (int u = 0; u < PER_PAIR; ++u) {
            bad[u] = q[u] > n;
            load_pair_half(lines, bad[u] ? 0 : q[u], hf, ph[u]);
            s[u] = reinterpret_cast<const uint4 *>(super)[ph[u].j / QR_LINES_PER_SB];
        }
#pragma unroll
        for (int u = 0; u < PER_PAIR; ++u) {
            uint32_t cnt[4];
            pair_count4(ph[u], hf, cnt);
            uint64_t r[4];
#pragma unroll
            for (uint32_t cc = 0; cc < 4; ++cc) {
                const uint64_t mine = hf == 0 ? ((uint64_t)sel4(s[u], cc) << QR_SHIFT) + pair_delta(ph[u], cc) - cnt[cc]
                                              : (uint64_t)cnt[cc];
                r[cc] = mine + pair_swap64(mine);
            }
            // lane 0 writes symbols A, C and lane 1 writes G, T of the row
            ra[u] = bad[u] ? ~0ull : (hf == 0 ? r[0] : r[2]);
            rb[u] = bad[u] ? ~0ull : (hf == 0 ? r[1] : r[3]);
        }
#pragma unroll
        for (int u = 0; u < PER_PAIR; ++u) {
            const uint64_t i = i0 + u * pairs;
            if (i < nq) {
                reinterpret_cast<ulonglong2 *>(out4 + 4 * i)[hf] = make_ulonglong2(ra[u], rb[u]);
                if (bad[u] && hf == 0) atomicOr(err, 1u);
            }
        }
    }
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

}  // namespace

namespace qr {

// Build the QuadRank layout into caller-provided arrays (also used by the FM-index build).
int quadrank_build_into(const uint64_t *d_packed2, uint64_t n, uint64_t *lines, uint32_t *super, hipStream_t stream) {
    const uint64_t n_lines = n / QR_DATA_BASES + 1, n_sb = n / QR_SB_BASES + 1, n_words = (n + 31) / 32;
    uint32_t *cnt = nullptr;
    uint64_t *base = nullptr;
    if (hipMalloc(&cnt, n_sb * 16) != hipSuccess || hipMalloc(&base, n_sb * 32) != hipSuccess) {
        (void)hipGetLastError();
        if (cnt) (void)hipFree(cnt);
        set_error("quadrank build: temporary allocation failed");
        return QR_ENOMEM;
    }
    hipLaunchKernelGGL(qr_count_kernel, dim3((uint32_t)n_sb), dim3(256), 0, stream, d_packed2, n, n_words, cnt);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = launch_scan_counts(cnt, n_sb, 4, QR_SHIFT, base, super, stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(qr_write_kernel, dim3((uint32_t)n_sb), dim3(128), 0, stream, d_packed2, n, n_words, base,
                           n_lines, lines);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    (void)hipFree(cnt);
    (void)hipFree(base);
    if (e != hipSuccess) {
        set_error("quadrank build: %s", hipGetErrorString(e));
        return QR_EHIP;
    }
    return QR_OK;
}

}  // namespace qr

extern "C" {

int quadrank_build(const uint64_t *d_packed2, uint64_t n, hipStream_t stream, qr_quadrank *out) {
    if (!out) {
        set_error("quadrank_build: out is NULL");
        return QR_EINVAL;
    }
    *out = nullptr;
    if (((uintptr_t)d_packed2 & 7) || (!d_packed2 && n)) {
        set_error("quadrank_build: d_packed2 is NULL with n = %llu", (unsigned long long)n);
        return QR_EINVAL;
    }
    if (n > QR_MAX_N) {
        set_error("quadrank_build: n = %llu exceeds the layout limit 2^44 - 1", (unsigned long long)n);
        return QR_ERANGE;
    }
    qr_quadrank_s *h = new (std::nothrow) qr_quadrank_s{};
    if (!h) return QR_ENOMEM;
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return QR_EHIP;
    }
    h->n = n;
    h->n_lines = n / QR_DATA_BASES + 1;
    h->n_sb = n / QR_SB_BASES + 1;
    h->tune = qr_tuning{256, 1, 0, 2};
    if (hipMalloc(&h->lines, h->n_lines * 128) != hipSuccess || hipMalloc(&h->super, h->n_sb * 16) != hipSuccess ||
        hipMalloc(&h->err, 4) != hipSuccess) {
        (void)hipGetLastError();
        set_error("quadrank_build: device allocation of %llu bytes failed",
                  (unsigned long long)(h->n_lines * 128 + h->n_sb * 16));
        release(h);
        return QR_ENOMEM;
    }
    if (hipMemsetAsync(h->err, 0, 4, stream) != hipSuccess) {
        release(h);
        return QR_EHIP;
    }
    int rc = quadrank_build_into(d_packed2, n, h->lines, h->super, stream);
    if (rc) {
        release(h);
        return rc;
    }
    *out = h;
    return QR_OK;
}

static int qr_launch_common(qr_quadrank h, uint64_t nq, const void *a, const void *b, const char *what) {
    if (!h || (nq && (!a || !b))) {
        set_error("%s: null handle or pointer", what);
        return QR_EINVAL;
    }
    if (((uintptr_t)a & 7) || ((uintptr_t)b & 15)) {
        set_error("%s: d_q must be 8-byte and the output 16-byte aligned", what);
        return QR_EINVAL;
    }
    return check_device(h->device);
}

int quadrank_rank(qr_quadrank h, const uint64_t *d_q, const uint8_t *d_c, uint64_t nq, uint64_t *d_out,
                  hipStream_t stream) {
    int rc = qr_launch_common(h, nq, d_q, d_out, "quadrank_rank");
    if (rc) return rc;
    if (nq && !d_c) {
        set_error("quadrank_rank: d_c is NULL");
        return QR_EINVAL;
    }
    if (!nq) return QR_OK;
    const int block = h->tune.block ? h->tune.block : 256, pl = h->tune.per_lane ? h->tune.per_lane : 1;
    const int lanes = h->tune.lanes == 1 ? 1 : 2;
    const dim3 g((uint32_t)grid_for(nq, pl, block, h->tune.grid_waves, lanes)), b(block);
    const uint4 *L = reinterpret_cast<const uint4 *>(h->lines);
    if (lanes == 2) {
        switch (pl) {
            case 1: hipLaunchKernelGGL(qr_rank1_pair_kernel<1>, g, b, 0, stream, L, h->super, h->n, d_q, d_c, nq, d_out, h->err); break;
            case 2: hipLaunchKernelGGL(qr_rank1_pair_kernel<2>, g, b, 0, stream, L, h->super, h->n, d_q, d_c, nq, d_out, h->err); break;
            case 4: hipLaunchKernelGGL(qr_rank1_pair_kernel<4>, g, b, 0, stream, L, h->super, h->n, d_q, d_c, nq, d_out, h->err); break;
            default: hipLaunchKernelGGL(qr_rank1_pair_kernel<8>, g, b, 0, stream, L, h->super, h->n, d_q, d_c, nq, d_out, h->err); break;
        }
        QR_HIP(hipGetLastError());
        return QR_OK;
    }
    switch (pl) {
        case 1: hipLaunchKernelGGL(qr_rank1_kernel<1>, g, b, 0, stream, L, h->super, h->n, d_q, d_c, nq, d_out, h->err); break;
        case 2: hipLaunchKernelGGL(qr_rank1_kernel<2>, g, b, 0, stream, L, h->super, h->n, d_q, d_c, nq, d_out, h->err); break;
        case 4: hipLaunchKernelGGL(qr_rank1_kernel<4>, g, b, 0, stream, L, h->super, h->n, d_q, d_c, nq, d_out, h->err); break;
        default: hipLaunchKernelGGL(qr_rank1_kernel<8>, g, b, 0, stream, L, h->super, h->n, d_q, d_c, nq, d_out, h->err); break;
    }
    QR_HIP(hipGetLastError());
    return QR_OK;
}

int quadrank_rank4(qr_quadrank h, const uint64_t *d_q, uint64_t nq, uint64_t *d_out4, hipStream_t stream) {
    int rc = qr_launch_common(h, nq, d_q, d_out4, "quadrank_rank4");
    if (rc) return rc;
    if (!nq) return QR_OK;
    const int block = h->tune.block ? h->tune.block : 256, pl = h->tune.per_lane ? h->tune.per_lane : 1;
    const int lanes = h->tune.lanes == 1 ? 1 : 2;
    const dim3 g((uint32_t)grid_for(nq, pl, block, h->tune.grid_waves, lanes)), b(block);
    const uint4 *L = reinterpret_cast<const uint4 *>(h->lines);
    if (lanes == 2) {
        switch (pl) {
            case 1: hipLaunchKernelGGL(qr_rank4_pair_kernel<1>, g, b, 0, stream, L, h->super, h->n, d_q, nq, d_out4, h->err); break;
            case 2: hipLaunchKernelGGL(qr_rank4_pair_kernel<2>, g, b, 0, stream, L, h->super, h->n, d_q, nq, d_out4, h->err); break;
            case 4: hipLaunchKernelGGL(qr_rank4_pair_kernel<4>, g, b, 0, stream, L, h->super, h->n, d_q, nq, d_out4, h->err); break;
            default: hipLaunchKernelGGL(qr_rank4_pair_kernel<8>, g, b, 0, stream, L, h->super, h->n, d_q, nq, d_out4, h->err); break;
        }
        QR_HIP(hipGetLastError());
        return QR_OK;
    }
    switch (pl) {
        case 1: hipLaunchKernelGGL(qr_rank4_kernel<1>, g, b, 0, stream, L, h->super, h->n, d_q, nq, d_out4, h->err); break;
        case 2: hipLaunchKernelGGL(qr_rank4_kernel<2>, g, b, 0, stream, L, h->super, h->n, d_q, nq, d_out4, h->err); break;
        case 4: hipLaunchKernelGGL(qr_rank4_kernel<4>, g, b, 0, stream, L, h->super, h->n, d_q, nq, d_out4, h->err); break;
        default: hipLaunchKernelGGL(qr_rank4_kernel<8>, g, b, 0, stream, L, h->super, h->n, d_q, nq, d_out4, h->err); break;
    }
    QR_HIP(hipGetLastError());
    return QR_OK;
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
uint64_t quadrank_bytes(qr_quadrank h) { return h ? h->n_lines * 128 + h->n_sb * 16 : 0; }

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
    if (h_super) QR_HIP(hipMemcpy(h_super, h->super, h->n_sb * 16, hipMemcpyDeviceToHost));
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
    h->tune = *t;
    if (!h->tune.lanes) h->tune.lanes = 2;
    return QR_OK;
}

}  // extern "C"
