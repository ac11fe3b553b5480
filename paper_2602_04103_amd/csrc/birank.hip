// BiRank on gfx950 (paper Section 3): binary rank with one 16-bit delta inlined per 128-byte line.
//
// Line j (16 little-endian u64 words = 1024 bits):
//   bits [0, 16)      b_j = rank(1008 j + 496) - 2^10 * s_{j/64}   (delta to the line's middle)
//   bits [16, 1024)   input bits [1008 j, 1008 j + 1008)
// The line's middle is line bit 512 (= data bit 496), so each half line is one 64-byte segment.
// Superblock i = lines [64 i, 64 i + 64) = 64512 input bits = exactly 1008 input words;
//   s_i = floor(rank(64512 i) / 2^10) as u32 (the paper's shifted 32-bit offset, Section 3,
//   with shift 10 instead of 11 because 64 lines of 1008 bits fill the 16-bit delta).
// Bound: b_j <= 63*1008 + 496 + (2^10 - 1) = 65023 < 2^16; s_i < 2^32 for n < 2^42.
// There are floor(n/1008) + 1 lines and floor(n/64512) + 1 superblocks, so q = n always has a
// line; bits past n are stored as zero and every delta is taken over that zero-padded text.
//
// Query (paper Eq. (1)): j = floor(q/1008), p = q - 1008 j + 16 (line bit of q);
//   rank(q) = 2^10 s_{j/64} + b_j + popcount(line bits [512, p))   if p >= 512
//   rank(q) = 2^10 s_{j/64} + b_j - popcount(line bits [p, 512))   if p <  512
// so at most one 64-byte half line (512 bits) is popcounted.
#include <algorithm>
#include <new>

#include "common.hpp"

using namespace qr;

struct qr_birank_s {
    int device;
    uint64_t n, n_lines, n_sb;
    uint64_t *lines;  // n_lines * 16 words
    uint32_t *super;  // n_sb
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

// Pass 1: number of 1 bits in each superblock (1008 consecutive input words).
__global__ __launch_bounds__(256) void br_count_kernel(const uint64_t *__restrict__ bits, uint64_t n,
                                                       uint64_t n_words, uint32_t *__restrict__ cnt) {
    const uint64_t sb = blockIdx.x;
    const uint64_t w0 = sb * (BR_SB_BITS / 64);
    uint32_t c = 0;
    for (uint32_t k = threadIdx.x; k < BR_SB_BITS / 64; k += 256) c += __popcll(masked_word(bits, w0 + k, n, n_words));
    c = wave_sum(c);
    __shared__ uint32_t part[4];
    if (__lane_id() == 0) part[threadIdx.x / 64] = c;
    __syncthreads();
    if (threadIdx.x == 0) cnt[sb] = part[0] + part[1] + part[2] + part[3];
}

// Pass 3: one 64-lane workgroup per superblock; lane t forms line 64 i + t.
constexpr int OUT_STRIDE = 17;  // padded LDS row (u64) for the staged lines: avoids bank conflicts

__global__ __launch_bounds__(64) void br_write_kernel(const uint64_t *__restrict__ bits, uint64_t n, uint64_t n_words,
                                                      const uint64_t *__restrict__ base, uint64_t n_lines,
                                                      uint64_t *__restrict__ lines) {
    constexpr int W = BR_SB_BITS / 64;  // 1008 input words
    __shared__ uint64_t in[W + 2];
    __shared__ uint64_t stage[64 * OUT_STRIDE];
    const uint64_t sb = blockIdx.x;
    const int t = threadIdx.x;
    for (int k = t; k < W + 2; k += 64) in[k] = k < W ? masked_word(bits, sb * W + k, n, n_words) : 0ull;
    __syncthreads();

    auto get64 = [&](uint32_t b) -> uint64_t {  // input bits [b, b+64) of this superblock
        uint32_t w = b >> 6, sh = b & 63;
        uint64_t lo = in[w];
        return sh ? (lo >> sh) | (in[w + 1] << (64 - sh)) : lo;
    };
    const uint32_t b0 = (uint32_t)BR_DATA_BITS * (uint32_t)t;
    uint64_t o[16];
    o[0] = get64(b0) << BR_HDR;
#pragma unroll
    for (int k = 1; k < 16; ++k) o[k] = get64(b0 + 64u * k - BR_HDR);
    uint32_t c_first = 0, c_second = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) c_first += __popcll(o[k]);
#pragma unroll
    for (int k = 8; k < 16; ++k) c_second += __popcll(o[k]);
    const uint32_t c_tot = c_first + c_second;
    const uint32_t before = wave_inclusive_scan<uint32_t>(c_tot) - c_tot;
    const uint32_t rem = (uint32_t)(base[sb] & ((1u << BR_SHIFT) - 1u));
    o[0] |= (uint64_t)(rem + before + c_first);
#pragma unroll
    for (int k = 0; k < 16; ++k) stage[t * OUT_STRIDE + k] = o[k];
    __syncthreads();
    const uint64_t l0 = sb * BR_LINES_PER_SB;
    const uint32_t nl = (uint32_t)std::min<uint64_t>(BR_LINES_PER_SB, n_lines - l0);
    uint4 *dst = reinterpret_cast<uint4 *>(lines + l0 * 16);
    for (uint32_t e = t; e < nl * 8; e += 64) {  // 8 uint4 per line, coalesced
        const uint64_t *src = stage + (e >> 3) * OUT_STRIDE + (e & 7) * 2;
        uint64_t a = src[0], b = src[1];
        dst[e] = make_uint4((uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32));
    }
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

// Query kernel: PER_LANE independent queries per lane, all loads issued before any popcount.
template <int PER_LANE>
__global__ __launch_bounds__(256) void br_rank_kernel(const uint4 *__restrict__ lines, const uint32_t *__restrict__ super,
                                                      uint64_t n, const uint64_t *__restrict__ Q, uint64_t nq,
                                                      uint64_t *__restrict__ out, uint32_t *__restrict__ err) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i0 < nq; i0 += stride * PER_LANE) {
        uint64_t q[PER_LANE], j[PER_LANE];
        uint32_t p[PER_LANE], hdr[PER_LANE], s[PER_LANE];
        uint32_t h[PER_LANE][16];
        bool bad[PER_LANE];
#pragma unroll
        for (int u = 0; u < PER_LANE; ++u) {
            const uint64_t i = i0 + u * stride;
            q[u] = i < nq ? Q[i] : 0;
            bad[u] = q[u] > n;
            if (bad[u]) q[u] = 0;  // line 0 always exists; the output is overwritten below
        }
#pragma unroll
        for (int u = 0; u < PER_LANE; ++u) {
            j[u] = br_line_of(q[u]);
            p[u] = (uint32_t)(q[u] - j[u] * BR_DATA_BITS) + BR_HDR;
            const bool up = p[u] >= BR_MID;
            const uint4 *L = lines + j[u] * 8 + (up ? 4 : 0);
            uint4 a = L[0], b = L[1], c = L[2], d = L[3];
            h[u][0] = a.x, h[u][1] = a.y, h[u][2] = a.z, h[u][3] = a.w;
            h[u][4] = b.x, h[u][5] = b.y, h[u][6] = b.z, h[u][7] = b.w;
            h[u][8] = c.x, h[u][9] = c.y, h[u][10] = c.z, h[u][11] = c.w;
            h[u][12] = d.x, h[u][13] = d.y, h[u][14] = d.z, h[u][15] = d.w;
            hdr[u] = up ? reinterpret_cast<const uint32_t *>(lines)[j[u] * 32] : a.x;
            s[u] = super[j[u] / BR_LINES_PER_SB];
        }
#pragma unroll
        for (int u = 0; u < PER_LANE; ++u) {
            const uint64_t i = i0 + u * stride;
            if (i >= nq) continue;
            const bool up = p[u] >= BR_MID;
            const uint32_t cnt = half_count(h[u], up ? p[u] - BR_MID : p[u], up);
            const uint64_t mid = ((uint64_t)s[u] << BR_SHIFT) + (hdr[u] & 0xffffu);
            uint64_t r = up ? mid + cnt : mid - cnt;
            if (bad[u]) {
                r = ~0ull;
                atomicOr(err, 1u);
            }
            out[i] = r;
        }
    }
}

// Lane-pair query kernel: lanes 2k and 2k+1 serve the same query; lane h loads half h (64 bytes)
// of the line, so every load instruction of a wave touches 32 lines with 64 contiguous bytes
// each (measured on MI355X: far fewer address-translation misses on multi-GiB structures than one
// lane issuing four loads).  The lane holding the half that contains q popcounts it; lane 0 adds
// the superblock offset and delta; the two contributions are summed across the pair.
template <int PER_PAIR>
__global__ __launch_bounds__(256) void br_rank_pair_kernel(const uint4 *__restrict__ lines,
                                                           const uint32_t *__restrict__ super, uint64_t n,
                                                           const uint64_t *__restrict__ Q, uint64_t nq,
                                                           uint64_t *__restrict__ out, uint32_t *__restrict__ err) {
    const uint32_t hf = threadIdx.x & 1u;
    const uint64_t pairs = ((uint64_t)gridDim.x * blockDim.x) >> 1;
    for (uint64_t i0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 1; i0 < nq; i0 += pairs * PER_PAIR) {
        uint64_t q[PER_PAIR], r[PER_PAIR];
        uint32_t p[PER_PAIR], s[PER_PAIR];
        uint32_t h[PER_PAIR][16];
        bool bad[PER_PAIR];
        // 1: query positions (index clamped so every load is unconditional and in bounds)
#pragma unroll
        for (int u = 0; u < PER_PAIR; ++u) q[u] = Q[min(i0 + u * pairs, nq - 1)];
        // 2: this lane's half line and the superblock offset
#pragma unroll
        for (int u = 0; u < PER_PAIR; ++u) {
            bad[u] = q[u] > n;
            const uint64_t qq = bad[u] ? 0 : q[u];
            const uint64_t j = br_line_of(qq);
            p[u] = (uint32_t)(qq - j * BR_DATA_BITS) + BR_HDR;
            const uint4 *L = lines + j * 8 + hf * 4;
            const uint4 a = L[0], b = L[1], c = L[2], d = L[3];
            h[u][0] = a.x, h[u][1] = a.y, h[u][2] = a.z, h[u][3] = a.w;
            h[u][4] = b.x, h[u][5] = b.y, h[u][6] = b.z, h[u][7] = b.w;
            h[u][8] = c.x, h[u][9] = c.y, h[u][10] = c.z, h[u][11] = c.w;
            h[u][12] = d.x, h[u][13] = d.y, h[u][14] = d.z, h[u][15] = d.w;
            s[u] = super[j / BR_LINES_PER_SB];
        }
        // 3: count and combine across the pair
#pragma unroll
        for (int u = 0; u < PER_PAIR; ++u) {
            const bool up = p[u] >= BR_MID;
            const uint32_t cnt = half_count(h[u], up ? p[u] - BR_MID : p[u], up) & (((uint32_t)up == hf) ? ~0u : 0u);
            const uint64_t mine = hf == 0 ? ((uint64_t)s[u] << BR_SHIFT) + (h[u][0] & 0xffffu) - cnt : (uint64_t)cnt;
            r[u] = bad[u] ? ~0ull : mine + pair_swap64(mine);
        }
        // 4: results
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

template <int PL>
hipError_t launch_rank_pair(const qr_birank_s *h, const uint64_t *d_q, uint64_t nq, uint64_t *d_out, hipStream_t s,
                            int block, int grid_waves) {
    const uint64_t lanes_needed = 2 * ((nq + PL - 1) / PL);
    uint64_t blocks = (lanes_needed + block - 1) / block;
    if (grid_waves > 0) blocks = std::min<uint64_t>(blocks, std::max<uint64_t>(1, (uint64_t)cu_count() * grid_waves * 64 / block));
    blocks = std::max<uint64_t>(1, std::min<uint64_t>(blocks, 0x7fffffffull));
    hipLaunchKernelGGL(br_rank_pair_kernel<PL>, dim3((uint32_t)blocks), dim3(block), 0, s,
                       reinterpret_cast<const uint4 *>(h->lines), h->super, h->n, d_q, nq, d_out, h->err);
    return hipGetLastError();
}

template <int PL>
hipError_t launch_rank(const qr_birank_s *h, const uint64_t *d_q, uint64_t nq, uint64_t *d_out, hipStream_t s,
                       int block, int grid_waves) {
    if (h->tune.lanes != 1) return launch_rank_pair<PL>(h, d_q, nq, d_out, s, block, grid_waves);
    uint64_t lanes_needed = (nq + PL - 1) / PL;
    uint64_t blocks = (lanes_needed + block - 1) / block;
    if (grid_waves > 0) {
        uint64_t cap = (uint64_t)cu_count() * grid_waves * 64 / block;
        if (cap < 1) cap = 1;
        blocks = std::min<uint64_t>(blocks, cap);
    }
    blocks = std::max<uint64_t>(1, std::min<uint64_t>(blocks, 0x7fffffffull));
    hipLaunchKernelGGL(br_rank_kernel<PL>, dim3((uint32_t)blocks), dim3(block), 0, s,
                       reinterpret_cast<const uint4 *>(h->lines), h->super, h->n, d_q, nq, d_out, h->err);
    return hipGetLastError();
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

int birank_build(const uint64_t *d_bits, uint64_t n, hipStream_t stream, qr_birank *out) {
    if (!out) {
        set_error("birank_build: out is NULL");
        return QR_EINVAL;
    }
    *out = nullptr;
    if (((uintptr_t)d_bits & 7) || (!d_bits && n)) {
        set_error("birank_build: d_bits is NULL with n = %llu", (unsigned long long)n);
        return QR_EINVAL;
    }
    if (n > BR_MAX_N) {
        set_error("birank_build: n = %llu exceeds the layout limit 2^42 - 1", (unsigned long long)n);
        return QR_ERANGE;
    }
    qr_birank_s *h = new (std::nothrow) qr_birank_s{};
    if (!h) return QR_ENOMEM;
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        set_error("hipGetDevice failed");
        return QR_EHIP;
    }
    h->n = n;
    h->n_lines = n / BR_DATA_BITS + 1;
    h->n_sb = n / BR_SB_BITS + 1;
    h->tune = qr_tuning{256, 1, 0, 2};
    const uint64_t n_words = (n + 63) / 64;
    uint32_t *cnt = nullptr;
    uint64_t *base = nullptr;
    auto fail = [&](int code) {
        if (cnt) (void)hipFree(cnt);
        if (base) (void)hipFree(base);
        release(h);
        return code;
    };
    if (hipMalloc(&h->lines, h->n_lines * 128) != hipSuccess || hipMalloc(&h->super, h->n_sb * 4) != hipSuccess ||
        hipMalloc(&h->err, 4) != hipSuccess || hipMalloc(&cnt, h->n_sb * 4) != hipSuccess ||
        hipMalloc(&base, h->n_sb * 8) != hipSuccess) {
        (void)hipGetLastError();
        set_error("birank_build: device allocation of %llu bytes failed",
                  (unsigned long long)(h->n_lines * 128 + h->n_sb * 16));
        return fail(QR_ENOMEM);
    }
    if (hipMemsetAsync(h->err, 0, 4, stream) != hipSuccess) return fail(QR_EHIP);
    hipLaunchKernelGGL(br_count_kernel, dim3((uint32_t)h->n_sb), dim3(256), 0, stream, d_bits, n, n_words, cnt);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = launch_scan_counts(cnt, h->n_sb, 1, BR_SHIFT, base, h->super, stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(br_write_kernel, dim3((uint32_t)h->n_sb), dim3(64), 0, stream, d_bits, n, n_words, base,
                           h->n_lines, h->lines);
        e = hipGetLastError();
    }
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
    const int block = h->tune.block ? h->tune.block : 256;
    const int pl = h->tune.per_lane ? h->tune.per_lane : 1;
    hipError_t e;
    switch (pl) {
        case 1: e = launch_rank<1>(h, d_q, nq, d_out, stream, block, h->tune.grid_waves); break;
        case 2: e = launch_rank<2>(h, d_q, nq, d_out, stream, block, h->tune.grid_waves); break;
        case 4: e = launch_rank<4>(h, d_q, nq, d_out, stream, block, h->tune.grid_waves); break;
        default: e = launch_rank<8>(h, d_q, nq, d_out, stream, block, h->tune.grid_waves); break;
    }
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
uint64_t birank_bytes(qr_birank h) { return h ? h->n_lines * 128 + h->n_sb * 4 : 0; }

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
    if (h_super) QR_HIP(hipMemcpy(h_super, h->super, h->n_sb * 4, hipMemcpyDeviceToHost));
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
    h->tune = *t;
    if (!h->tune.lanes) h->tune.lanes = 2;
    return QR_OK;
}

}  // extern "C"
