// Random-line gather microbenchmark: the achievable throughput of one random 128-byte line (or a
// 64-byte half of one) per query, with the same per-query index read and result write as a rank
// query.  This is the measured ceiling the rank kernels are compared against.
#include <algorithm>

#include "common.hpp"

using namespace qr;

namespace {

template <int SEGS>  // 16-byte segments read per query: 4 (64 B) or 8 (128 B)
__global__ __launch_bounds__(256) void gather_kernel(const uint4 *__restrict__ lines, uint64_t n_lines,
                                                     const uint64_t *__restrict__ idx, uint64_t nq,
                                                     uint64_t *__restrict__ out) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nq) return;
    const uint64_t l = mulhi64(idx[i], n_lines);  // uniform line in [0, n_lines)
    const uint4 *L = lines + l * 8;
    uint4 v[SEGS];
#pragma unroll
    for (int k = 0; k < SEGS; ++k) v[k] = L[k];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < SEGS; ++k) s += v[k].x + v[k].y + v[k].z + v[k].w;
    out[i] = s;
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// LANES lanes share one query: lane t of the group reads 16-byte segments [t S, t S + S) of the line,
// S = 8 / LANES, and the group's sum is reduced across its lanes; the group's first lane writes it.
// NT: the line loads carry the non-temporal hint; IO: the index loads and result stores do.
template <int LANES, bool NT, bool IO>
__global__ __launch_bounds__(256) void gather_lanes_kernel(const uint4 *__restrict__ lines, uint64_t n_lines,
                                                           const uint64_t *__restrict__ idx, uint64_t nq,
                                                           uint64_t *__restrict__ out) {
    constexpr int S = 8 / LANES;
    const uint64_t g = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / LANES;
    const int t = threadIdx.x % LANES;
    const uint64_t i = g < nq ? g : nq - 1;  // whole groups stay active for the reduction
    const uint64_t l = mulhi64(IO ? load_once(idx + i) : idx[i], n_lines);
    const uint4 *L = lines + l * 8 + t * S;
    uint4 v[S];
#pragma unroll
    for (int k = 0; k < S; ++k) {
        if (NT) {
            const u32x4 x = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(L + k));
            v[k] = make_uint4(x.x, x.y, x.z, x.w);
        } else {
            v[k] = L[k];
        }
    }
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < S; ++k) s += v[k].x + v[k].y + v[k].z + v[k].w;
#pragma unroll
    for (int m = 1; m < LANES; m <<= 1) s += __shfl_xor(s, m, 64);
    if (t == 0 && g < nq) {
        if (IO)
            store_once(out + g, (uint64_t)s);
        else
            out[g] = s;
    }
}

}  // namespace

extern "C" int qr_gather_lanes_bench_ex(const void *d_lines, uint64_t n_lines, const uint64_t *d_idx, uint64_t nq,
                                        uint32_t lanes, uint32_t flags, uint64_t *d_out, hipStream_t stream) {
    if (!d_lines || !n_lines || (nq && (!d_idx || !d_out)) || (lanes != 1 && lanes != 2 && lanes != 4 && lanes != 8) ||
        (flags & ~(QR_GATHER_NONTEMPORAL | QR_GATHER_STREAM_IO)) || ((uintptr_t)d_lines & 15) || ((uintptr_t)d_idx & 7) ||
        ((uintptr_t)d_out & 7)) {
        set_error("qr_gather_lanes_bench: bad arguments");
        return QR_EINVAL;
    }
    if (!nq) return QR_OK;
    const uint64_t blocks = (nq * lanes + 255) / 256;
    if (blocks > 0x7fffffffull) {
        set_error("qr_gather_lanes_bench: nq too large");
        return QR_EINVAL;
    }
    const uint4 *L = reinterpret_cast<const uint4 *>(d_lines);
    const dim3 g((uint32_t)blocks), b(256);
#define QR_GL(N, T, I) hipLaunchKernelGGL((gather_lanes_kernel<N, T, I>), g, b, 0, stream, L, n_lines, d_idx, nq, d_out)
#define QR_GL2(N)                                   \
    if (nt) {                                       \
        if (io) QR_GL(N, true, true);               \
        else QR_GL(N, true, false);                 \
    } else {                                        \
        if (io) QR_GL(N, false, true);              \
        else QR_GL(N, false, false);                \
    }
    const bool nt = flags & QR_GATHER_NONTEMPORAL, io = flags & QR_GATHER_STREAM_IO;
    switch (lanes) {
        case 1: QR_GL2(1); break;
        case 2: QR_GL2(2); break;
        case 4: QR_GL2(4); break;
        default: QR_GL2(8); break;
    }
#undef QR_GL2
#undef QR_GL
    QR_HIP(hipGetLastError());
    return QR_OK;
}

extern "C" int qr_gather_lanes_bench(const void *d_lines, uint64_t n_lines, const uint64_t *d_idx, uint64_t nq,
                                     uint32_t lanes, uint64_t *d_out, hipStream_t stream) {
    return qr_gather_lanes_bench_ex(d_lines, n_lines, d_idx, nq, lanes, 0, d_out, stream);
}

extern "C" int qr_gather_bench(const void *d_lines, uint64_t n_lines, const uint64_t *d_idx, uint64_t nq,
                               uint32_t bytes_per_query, uint64_t *d_out, hipStream_t stream) {
    if (!d_lines || !n_lines || (nq && (!d_idx || !d_out)) || (bytes_per_query != 64 && bytes_per_query != 128) ||
        ((uintptr_t)d_lines & 15) || ((uintptr_t)d_idx & 7) || ((uintptr_t)d_out & 7)) {
        set_error("qr_gather_bench: bad arguments");
        return QR_EINVAL;
    }
    if (!nq) return QR_OK;
    const uint64_t blocks = (nq + 255) / 256;
    if (blocks > 0x7fffffffull) {
        set_error("qr_gather_bench: nq too large");
        return QR_EINVAL;
    }
    const uint4 *L = reinterpret_cast<const uint4 *>(d_lines);
    if (bytes_per_query == 64)
        hipLaunchKernelGGL(gather_kernel<4>, dim3((uint32_t)blocks), dim3(256), 0, stream, L, n_lines, d_idx, nq, d_out);
    else
        hipLaunchKernelGGL(gather_kernel<8>, dim3((uint32_t)blocks), dim3(256), 0, stream, L, n_lines, d_idx, nq, d_out);
    QR_HIP(hipGetLastError());
    return QR_OK;
}
