// Shared device helpers and host error plumbing for the rank library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdarg>
#include <cstdio>

#include "../../include/quadrank.h"

namespace qr {

// ---------------------------------------------------------------------------------------------
// Host error reporting: a per-thread message for qr_last_error().
void set_error(const char *fmt, ...);

#define QR_HIP(call)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess) {                                                                   \
            ::qr::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__,       \
                            __LINE__);                                                            \
            return QR_EHIP;                                                                       \
        }                                                                                         \
    } while (0)

// Returns QR_EINVAL unless the current device equals `dev`.
int check_device(int dev);

// Number of compute units of the current device (cached per device).
int cu_count();

// Build pass 2 (scan.hip): exclusive prefix sums of `ncol` interleaved u32 count columns.
hipError_t launch_scan_counts(const uint32_t *cnt, uint64_t nrow, int ncol, uint32_t shift, uint64_t *base,
                              uint32_t *super, hipStream_t s);

// ---------------------------------------------------------------------------------------------
// Exact floor division by the line payloads.  For a divisor d and shift s with
// m = ceil(2^s / d) and e = m*d - 2^s < d, floor(x*m / 2^s) = floor(x/d) holds for every
// x with x*e < 2^s (Granlund and Montgomery, PLDI 1994).  With s = 64 + t and m < 2^64 the
// quotient is the high word of the 128-bit product shifted right by t.
//   1008 (BiRank payload):  s = 73, e = 880 -> exact for x < 2^63
//    480 (QuadRank payload): s = 72, e = 224 -> exact for x < 2^63
// The BiRank constants live with its layout traits (birank_dev.hpp); the 16-bit QuadRank constants
// below are those of its trait QR16 (quadrank_dev.hpp).
constexpr uint64_t QR_DATA_BASES = 480;  // bases per QuadRank line
constexpr uint64_t QR_LINES_PER_SB = 128;
constexpr uint64_t QR_SB_BASES = QR_DATA_BASES * QR_LINES_PER_SB;  // 61440 = 1920 input words
constexpr uint32_t QR_SHIFT = 12;
constexpr uint32_t QR_MID = 256;         // line base position of the middle
constexpr uint32_t QR_HDR = 32;          // base slots taken by the four deltas
constexpr uint64_t QR_MAGIC = 0x8888888888888889ull;  // ceil(2^72 / 480)
constexpr uint32_t QR_MAGIC_T = 8;

__host__ __device__ __forceinline__ uint64_t mulhi64(uint64_t a, uint64_t b) {
    return (uint64_t)(((unsigned __int128)a * (unsigned __int128)b) >> 64);
}
__host__ __device__ __forceinline__ uint64_t qr_line_of(uint64_t q) { return mulhi64(q, QR_MAGIC) >> QR_MAGIC_T; }

// Mask selecting bit positions [0, t) of the 32-bit word that covers positions [32k, 32k+32).
__device__ __forceinline__ uint32_t prefix_mask32(uint32_t t, uint32_t k) {
    int32_t r = (int32_t)t - (int32_t)(32u * k);
    if (r <= 0) return 0u;
    if (r >= 32) return 0xffffffffu;
    return (1u << r) - 1u;
}

// Gather even bits (positions 0,2,..,62) of x into the low 32 bits (bit unshuffle).
__device__ __forceinline__ uint32_t even_bits(uint64_t x) {
    x &= 0x5555555555555555ull;
    x = (x | (x >> 1)) & 0x3333333333333333ull;
    x = (x | (x >> 2)) & 0x0f0f0f0f0f0f0f0full;
    x = (x | (x >> 4)) & 0x00ff00ff00ff00ffull;
    x = (x | (x >> 8)) & 0x0000ffff0000ffffull;
    x = (x | (x >> 16)) & 0x00000000ffffffffull;
    return (uint32_t)x;
}

// Inclusive prefix sum over the 64 lanes of a wavefront.
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
    const int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

// Value held by the other lane of this lane's pair (lane ^ 1), by a DPP quad permute [1,0,3,2].
__device__ __forceinline__ uint32_t pair_swap32(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, false);
}
__device__ __forceinline__ uint64_t pair_swap64(uint64_t x) {
    return (uint64_t)pair_swap32((uint32_t)x) | ((uint64_t)pair_swap32((uint32_t)(x >> 32)) << 32);
}

// Query batches and results stream through a rank launch once.  They are loaded and stored with the
// non-temporal hint, so they do not displace the structure's lines from L2 and from the memory-side
// cache (256 MB, a fifth of a 2^32-base QuadRank), whose hits on those lines lift the gather rate.
template <typename T>
__device__ __forceinline__ T load_once(const T *p) {
    return __builtin_nontemporal_load(p);
}
template <typename T>
__device__ __forceinline__ void store_once(T *p, T v) {
    __builtin_nontemporal_store(v, p);
}
typedef uint64_t u64x2_t __attribute__((ext_vector_type(2)));
// Two results to a 16-byte aligned address.
__device__ __forceinline__ void store_once2(uint64_t *p, uint64_t a, uint64_t b) {
    const u64x2_t v = {a, b};
    __builtin_nontemporal_store(v, reinterpret_cast<u64x2_t *>(p));
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

}  // namespace qr
