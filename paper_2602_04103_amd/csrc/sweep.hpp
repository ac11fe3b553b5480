// Position-ordered query tiles ("sweep" launch form of the rank kernels).
//
// A workgroup takes a tile of up to 256*QPT consecutive queries, counting-sorts them in LDS into
// SWEEP_BUCKETS buckets by the top bits of the position, and answers them in bucket order.  All
// resident workgroups start together and walk their tiles from low to high positions at about the
// same pace, so the loads in flight at any moment fall in a narrow band of the structure instead of
// the whole of it: fewer translation misses and more DRAM row hits per line.  Results go to the
// queries' own output slots, so the order is invisible to the caller; each answer is a function of
// its query alone, so the (racy) order inside a bucket does not change any output.
#pragma once

#include "common.hpp"

namespace qr {

constexpr int SWEEP_BLOCK = 256;
constexpr uint32_t SWEEP_BUCKETS = 256;

// Tile sizes of the sweep form and the settings it supports (lane pairs, 1 or 2 queries per pair).
__host__ __forceinline__ bool sweep_tuning_ok(const qr_tuning *t) {
    if (!t->sweep) return true;
    if (t->sweep != 1024 && t->sweep != 2048 && t->sweep != 4096) return false;
    return (t->lanes == 0 || t->lanes == 2) && (t->per_lane == 0 || t->per_lane == 1 || t->per_lane == 2);
}

// Whether a launch takes the sweep form: it is selected and its one-tile-per-workgroup grid fits
// the grid limit (otherwise the plain grid-stride form answers, with the same results).
__host__ __forceinline__ bool sweep_fits(int32_t sweep, uint64_t nq) {
    return sweep > 0 && (nq + (uint64_t)sweep - 1) / (uint64_t)sweep <= 0x7fffffffull;
}

// Right shift that maps every valid position q <= n to a bucket below 256.
__host__ __forceinline__ uint32_t sweep_shift(uint64_t n) {
    uint32_t bits = 0;
    while (bits < 64 && (n >> bits)) ++bits;  // bit length of n
    return bits > 8 ? bits - 8 : 0;
}

// LDS of one tile.  q holds the sorted positions and, for the rank rows, is overwritten in place by
// the results; slot_of[i] is the sorted slot of tile query i and tile_of[s] its inverse.
template <int QPT, bool HAS_C>
struct SweepLds {
    uint64_t q[SWEEP_BLOCK * QPT];
    uint16_t slot_of[SWEEP_BLOCK * QPT];
    uint16_t tile_of[SWEEP_BLOCK * QPT];
    uint8_t c[HAS_C ? SWEEP_BLOCK * QPT : 1];
    uint32_t start[SWEEP_BUCKETS];
};

// Exclusive scan of the 256 bucket counts in place, by the first wave (four counts per lane).
__device__ __forceinline__ void sweep_scan_buckets(uint32_t *start) {
    const uint32_t t = threadIdx.x;
    if (t < 64) {
        const uint32_t v0 = start[4 * t], v1 = start[4 * t + 1], v2 = start[4 * t + 2], v3 = start[4 * t + 3];
        const uint32_t sum = v0 + v1 + v2 + v3;
        uint32_t incl = sum;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t o = __shfl_up(incl, d, 64);
            if ((int)t >= d) incl += o;
        }
        const uint32_t ex = incl - sum;
        start[4 * t] = ex;
        start[4 * t + 1] = ex + v0;
        start[4 * t + 2] = ex + v0 + v1;
        start[4 * t + 3] = ex + v0 + v1 + v2;
    }
}

// Load the m (<= 256*QPT) queries of the tile starting at query `base` and leave them sorted by
// bucket in S.q (and S.c).  Ends with a barrier.
template <int QPT, bool HAS_C>
__device__ __forceinline__ void sweep_sort(const uint64_t *__restrict__ Q, const uint8_t *__restrict__ Cs, uint64_t base,
                                           uint32_t m, uint32_t shift, SweepLds<QPT, HAS_C> &S) {
    const uint32_t t = threadIdx.x;
    for (uint32_t b = t; b < SWEEP_BUCKETS; b += SWEEP_BLOCK) S.start[b] = 0;
    __syncthreads();
    uint64_t q[QPT];
    uint32_t key[QPT];  // bucket << 16 | rank inside the bucket
    uint32_t c[QPT];
#pragma unroll
    for (int k = 0; k < QPT; ++k) {
        const uint32_t i = k * SWEEP_BLOCK + t;
        if (i < m) {
            q[k] = load_once(Q + base + i);
            c[k] = HAS_C ? load_once(Cs + base + i) : 0u;
            const uint64_t hi = q[k] >> shift;
            const uint32_t b = hi < SWEEP_BUCKETS ? (uint32_t)hi : SWEEP_BUCKETS - 1;  // q > n: last bucket
            key[k] = b << 16 | atomicAdd(&S.start[b], 1u);
        }
    }
    __syncthreads();
    sweep_scan_buckets(S.start);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < QPT; ++k) {
        const uint32_t i = k * SWEEP_BLOCK + t;
        if (i < m) {
            const uint32_t s = S.start[key[k] >> 16] + (key[k] & 0xffffu);
            S.q[s] = q[k];
            if (HAS_C) S.c[s] = (uint8_t)c[k];
            S.slot_of[i] = (uint16_t)s;
            S.tile_of[s] = (uint16_t)i;
        }
    }
    __syncthreads();
}

// Write the tile's results, left in S.q in sorted order, to out[base + i] in query order.
template <int QPT, bool HAS_C>
__device__ __forceinline__ void sweep_store(uint64_t *__restrict__ out, uint64_t base, uint32_t m,
                                            const SweepLds<QPT, HAS_C> &S) {
#pragma unroll
    for (int k = 0; k < QPT; ++k) {
        const uint32_t i = k * SWEEP_BLOCK + threadIdx.x;
        if (i < m) store_once(out + base + i, S.q[S.slot_of[i]]);
    }
}

}  // namespace qr
